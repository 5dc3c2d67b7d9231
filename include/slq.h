/*
 * slq.h - C ABI of libslq, the MI355X (gfx950) hot path of self-learning
 * determinantal quantum Monte Carlo (Xu, Qi, Liu, Fu, Meng, arXiv:1612.03804).
 *
 * Notation (paper, "Basics of DQMC", Eq. 1):
 *   lattice        periodic lx x ly square lattice, N = lx*ly, site i = x + lx*y
 *   slices         l = 1..L imaginary-time slices, L*dtau = beta
 *   field          s_{i,l} = +-1, stored int8 s[l-1][i] (slice-major)
 *   kinetic        K_ij = -t on nearest-neighbour bonds (a length-2 dimension
 *                  carries the bond twice), K_ii = -mu;  E = exp(-dtau K)
 *   slice matrix   B_l = E diag(exp(-dtau xi s_{.,l}))
 *   weight         W_f(s) = det(1 + B_L ... B_1)    (fermion determinant of Eq. 1)
 *   Green's fn.    G = (1 + B_L ... B_1)^{-1},  G[i][j] = <c_i c_j^dag>, row-major
 *
 * Conventions shared by every call:
 *   - Return value: SLQ_OK or a negative SLQ_ERR_* code; slq_last_error()
 *     returns a thread-local message for the last failure.  Nothing throws.
 *   - Pointers named d_* are device pointers owned by the caller; the library
 *     never frees or retains them past the call.  Pointers without d_ are host
 *     pointers, read during the call only.
 *   - Calls are asynchronous on the caller's HIP stream `stream` (0 = the null
 *     stream): host-side argument checks return at once; everything else is
 *     enqueued.  Results are valid after the caller synchronises the stream.
 *   - Per-item problems found on the device (a spin that is not +-1, a
 *     non-finite intermediate, a singular final matrix) are written to
 *     d_status[b] (0 = ok, SLQ_ST_* bits otherwise) and do not abort the batch.
 *   - A plan (slq_plan) owns device workspace sized for one model and a
 *     maximum batch; it is created and destroyed on the host (allocation and
 *     release are synchronous).  Calls on one plan must not overlap in time:
 *     they share its workspace.  Distinct plans are independent.
 *   - Random numbers: Philox4x64-10 (Salmon et al., SC'11), key (seed, tag),
 *     4-word counter chosen per decision as documented per call; uniform
 *     u = (word0 >> 11) * 2^-53, integer in [0,n) = ((word0 >> 32) * n) >> 32.
 *     Chain index = chain0 + batch position.
 */
#ifndef SLQ_H
#define SLQ_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SLQ_OK = 0,
  SLQ_ERR_ARG = -1,       /* invalid argument (sizes, null pointers, unusable terms) */
  SLQ_ERR_DEVICE = -2,    /* no HIP device, or a HIP runtime call failed */
  SLQ_ERR_WORKSPACE = -3, /* batch larger than the plan was created for */
  SLQ_ERR_NUMERIC = -4    /* host-visible numeric failure (fit: singular normal equations) */
};

/* d_status bits */
enum {
  SLQ_ST_BAD_SPIN = 1,    /* a field entry is not +-1 */
  SLQ_ST_NONFINITE = 2,   /* a non-finite value appeared in the stabilised chain */
  SLQ_ST_SINGULAR = 4,    /* the final matrix M has a zero pivot (W_f = 0) */
  SLQ_ST_PIVOT = 8        /* internal check: an LU pivot index outside the rows below the
                             diagonal was refused (that interchange skipped); not expected */
};

/* How the chain product X <- E diag(d_l) X is formed.  The QR/UDV
 * stabilisation, the final LU, log-det and G are FP64 in every mode.
 * SLQ_PREC_FP64: FP64, using that E = e^{dtau mu} Cx (x) Cy is a Kronecker
 *   product of two circulants on the periodic lattice (lattice lines along x,
 *   then along y: 2N^2 (lx+ly) flops per slice and field instead of 2N^3;
 *   lattices with lx or ly > 64 fall back to the dense FP64 product).
 * SLQ_PREC_FP64_DENSE: FP64 dense GEMMs with E on the matrix cores.
 * SLQ_PREC_FP32 / SLQ_PREC_BF16: dense GEMMs with E and X rounded to the
 *   operand type at every GEMM, FP32 accumulation on the matrix cores, X kept
 *   in FP32 between slices.
 * SLQ_PREC_CHECKERBOARD: FP64 with the checkerboard split in place of E
 *   (the sparse slice matrices behind the beta N^2 chain cost of "Formalism of
 *   SLDQMC"): the bonds of the torus in four groups of disjoint bonds, x bonds
 *   from even / odd x (A / B) and y bonds from even / odd y (C / D), and
 *   E_cb = e^{dtau mu} A' B' C' D C' B' A' with X' the half-step factor
 *   exp(-dtau K_X / 2) (a 2 x 2 rotation cosh + sinh sigma_x on each bond).
 *   A different discretisation of the same model: E_cb - E = O(dtau^3), so the
 *   weight differs from SLQ_PREC_FP64's by O(dtau^2) at fixed beta.  22 N
 *   flops per vector and slice.  Needs even lx and ly (else SLQ_ERR_ARG);
 *   slq_kinetic returns E_cb and E_cb^{-1}, and every product of the plan
 *   (chains, local sweeps, bilayer, measurements) uses them. */
enum {
  SLQ_PREC_FP64 = 0,
  SLQ_PREC_FP32 = 1,
  SLQ_PREC_BF16 = 2,
  SLQ_PREC_FP64_DENSE = 3,
  SLQ_PREC_CHECKERBOARD = 4
};

typedef struct slq_model {
  int32_t lx, ly;      /* lattice extents, >= 1 each, N = lx*ly <= 2400 */
  int32_t n_slices;    /* L >= 1 */
  int32_t n_stab;      /* slices multiplied between QR stabilisations, >= 1 */
  double t, mu;        /* hopping and chemical potential */
  double dtau, xi;     /* slice width (> 0) and Ising-fermion coupling */
  int32_t chain_prec;  /* SLQ_PREC_*: operand precision of the chain GEMMs */
} slq_model;

typedef struct slq_plan slq_plan;
typedef struct slq_eff slq_eff; /* an effective model on a plan: see slq_eff_create */

/* Library version string and the last error message of this thread. */
const char* slq_version(void);
const char* slq_last_error(void);

/*
 * Plans.  A plan holds the device workspace for `model` and up to `max_batch`
 * simultaneous fields: E = exp(-dtau K) and E^{-1} (built there from the
 * closed form: K is diagonal in lattice momentum, so E is e^{dtau mu} times
 * the Kronecker product of two circulant 1-D propagators; model definition:
 * "Basics of DQMC", B^tau = exp(dtau K) exp(V), with the sign conventions at
 * the top of this header), the chain and factorisation buffers, and, by
 * flag, the buffers of local sweeps and of the learned action.  No call on a
 * plan allocates device memory afterwards.
 *
 * Flags: SLQ_PLAN_SWEEPS adds the stacked partial products of
 * slq_sweep_local ((floor((L-1)/n_stab) + 1) * max_batch * (2N^2 + N)
 * doubles); SLQ_PLAN_NET adds the activations of the network calls
 * (6 * 8 * L * N * max_batch doubles and small per-field arrays).  Calls that
 * need a section the plan was created without return SLQ_ERR_WORKSPACE.
 *
 * slq_plan_workspace_size - *bytes = the workspace size for (model,
 * max_batch, flags).  Host only.
 * slq_plan_create - create the plan on the current HIP device.  With d_work
 * != NULL the plan lives in that caller-owned device memory (256-byte
 * aligned, at least the queried size; the caller frees it after
 * slq_plan_destroy) and the library allocates nothing; with d_work == NULL
 * the plan allocates the workspace once, here, and frees it in
 * slq_plan_destroy.  Synchronous (E is built before it returns).  *out
 * receives the plan.  Errors: SLQ_ERR_ARG (sizes, flags, alignment),
 * SLQ_ERR_WORKSPACE (work_bytes too small), SLQ_ERR_DEVICE.
 */
enum { SLQ_PLAN_SWEEPS = 1, SLQ_PLAN_NET = 2 };
int slq_plan_workspace_size(const slq_model* model, int32_t max_batch, int32_t flags, size_t* bytes);
int slq_plan_create(const slq_model* model, int32_t max_batch, int32_t flags, void* d_work, size_t work_bytes,
                    slq_plan** out);
int slq_plan_destroy(slq_plan* plan);
/* Device bytes held by the plan. */
int slq_plan_bytes(const slq_plan* plan, size_t* bytes);

/* slq_plan_tune - time the admissible block widths (vectors per workgroup:
 * 2, 4, ..., 32) of the structured chain product (SLQ_PREC_FP64) on `batch`
 * fields of the plan's own workspace and keep the fastest for later calls;
 * *chosen (host, may be NULL) receives it.  Plans with dense FP64 chain
 * products (SLQ_PREC_FP64_DENSE) get the fastest tile shape of their chain
 * GEMM instead, and *chosen = 0; reduced-precision plans are left as they
 * are.  Synchronous on `stream`; overwrites the plan's scratch; must not run
 * during stream capture.  Without it the plan uses a width fixed by the LDS
 * size and a tile shape fixed by N. */
int slq_plan_tune(slq_plan* plan, int32_t batch, int32_t* chosen, hipStream_t stream);
/* slq_plan_set_block_width - fix the structured chain product's block width
 * (vectors per workgroup, a power of two 1..32 whose workgroup fits the
 * lattice: at most 1024 threads, 512 for sides above 24, and 160 KiB of LDS)
 * instead of tuning it; 0 returns to the width fixed by the LDS size.  Host
 * only, takes effect at the next call.  Results do not depend on the width
 * beyond rounding order.  Errors: SLQ_ERR_ARG (NULL plan, a plan with dense
 * products, an inadmissible width). */
int slq_plan_set_block_width(slq_plan* plan, int32_t width);
/* Copy E (or E^{-1} when inverse != 0) into caller memory d_out [N][N]. */
int slq_kinetic(slq_plan* plan, int32_t inverse, double* d_out, hipStream_t stream);

/*
 * Kernel timing of the three parts of every exact evaluation, on the call's
 * stream (Eq. 1's B(beta,0) as products of B^tau, then stabilised):
 *   SLQ_PROFILE_CHAIN   the chain products: one launch per block of n_stab
 *                       slices (structured FP64: 2 N^2 (lx+ly) flops per slice
 *                       and field) or per slice (dense GEMMs: 2 N^3);
 *   SLQ_PROFILE_STAB    each stabilisation: the QR of X diag(D) with its
 *                       explicit Q ((8/3) N^3 flops per field) and the V
 *                       update (N^3; none for the first block);
 *   SLQ_PROFILE_FINISH  the final step: with G an LU and two triangular
 *                       solves ((8/3) N^3), without G a QR of M ((4/3) N^3,
 *                       (2/3) N^3 where the LU serves, N <= 64).
 * The flop counts are algorithmic (what the factorisations need), not what
 * the kernels issue.  While enabled, HIP events are recorded around each
 * such sequence.  slq_profile_read_part waits for one part's events and
 * returns their summed duration in ms, the number of sequences and the
 * flops, then clears that part's record; slq_profile_read is the chain
 * part.  Enabling also clears the records.  Host-side only, synchronous.
 */
enum { SLQ_PROFILE_CHAIN = 0, SLQ_PROFILE_STAB = 1, SLQ_PROFILE_FINISH = 2 };
int slq_profile_enable(slq_plan* plan, int32_t enable);
int slq_profile_read(slq_plan* plan, double* ms, int64_t* launches, double* flops);
int slq_profile_read_part(slq_plan* plan, int32_t part, double* ms, int64_t* launches, double* flops);

/*
 * slq_weight - exact fermion weight of Eq. 1 for `batch` fields:
 *   d_logabs[b] = log|det(1 + B_L...B_1)|, d_sign[b] = sign (+1/-1, 0 if W_f = 0).
 * d_s: int8 [batch][L][N].  The chain is kept as U diag(D) V and refactored by
 * a column-pre-pivoted Householder QR every n_stab slices (the paper cites
 * the standard O(beta N^3) stabilised algorithm without describing it).
 * d_status: int32 [batch] (may be NULL).  Errors: SLQ_ERR_ARG,
 * SLQ_ERR_WORKSPACE (batch > max_batch), SLQ_ERR_DEVICE.
 */
int slq_weight(slq_plan* plan, int32_t batch, const int8_t* d_s,
               double* d_logabs, int8_t* d_sign, int32_t* d_status, hipStream_t stream);

/*
 * slq_weight_static - slq_weight without a plan and without allocating
 * anything, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * plan's workspace is laid out in a file-scope device array of
 * SLQ_STATIC_SCRATCH_BYTES, one per GPU the library runs on (held until the
 * process ends); E and E^{-1} are rebuilt in it on every call, nothing is
 * carried over from an earlier call.  Every call on one GPU shares that
 * array: calls that overlap in time on one GPU race (serialise them, e.g. on
 * one stream).  FP64 chains (SLQ_PREC_FP64, SLQ_PREC_FP64_DENSE,
 * SLQ_PREC_CHECKERBOARD) only.
 * Arguments and results as slq_weight, for `batch` fields of `model`.
 * Errors: SLQ_ERR_ARG, SLQ_ERR_WORKSPACE (the model and batch need more
 * than SLQ_STATIC_SCRATCH_BYTES: slq_plan_workspace_size with flags 0 tells
 * how much), SLQ_ERR_DEVICE.
 */
#define SLQ_STATIC_SCRATCH_BYTES (64u << 20)
int slq_weight_static(const slq_model* model, int32_t batch, const int8_t* d_s, double* d_logabs,
                      int8_t* d_sign, int32_t* d_status, hipStream_t stream);

/*
 * slq_green - as slq_weight, and also the equal-time Green's function
 * d_G[b] = (1 + B_L...B_1)^{-1}, FP64 [batch][N][N] row-major.
 */
int slq_green(slq_plan* plan, int32_t batch, const int8_t* d_s, double* d_G,
              double* d_logabs, int8_t* d_sign, int32_t* d_status, hipStream_t stream);

/*
 * slq_udv - the stabilised factorisation U diag(D) V of the cyclic chain that
 * starts at slice slice0 + 1:  B_{k(L)} ... B_{k(1)}, k(j) = (slice0 + j - 1)
 * mod L + 1 (slice0 = 0 gives B_L ... B_1).  U is orthogonal, D > 0 holds
 * the graded scales and V is well conditioned; the factorisation is the one
 * slq_weight/slq_green finish from.  d_U, d_V: FP64 [batch][N][N] row-major;
 * d_D: FP64 [batch][N].  0 <= slice0 < L.
 */
int slq_udv(slq_plan* plan, int32_t batch, const int8_t* d_s, int32_t slice0,
            double* d_U, double* d_D, double* d_V, int32_t* d_status, hipStream_t stream);

/*
 * slq_magnetization - d_M[b] = sum_{i,l} s_{i,l} (int64) of each field: the
 * total magnetisation whose autocorrelation C(t) over sweeps or cumulative
 * updates defines the autocorrelation time (Fig. 1 caption; tau_L in
 * "Basics of DQMC").  d_s int8 [batch][L][N].
 */
int slq_magnetization(slq_plan* plan, int32_t batch, const int8_t* d_s, int64_t* d_M, hipStream_t stream);

/*
 * slq_measure_equal_time - equal-time observables of each Green's function
 * d_G FP64 [batch][N][N] (G[i][j] = <c_i c_j^dag> as slq_green returns it;
 * for a given field the fermions are free, so Wick's theorem gives
 * <c_i^dag c_j> = delta_ij - G_ji and <n_i n_j> = (1 - G_ii)(1 - G_jj) +
 * (delta_ij - G_ji) G_ij).  d_out FP64 [batch][3]: the density
 * (1/N) sum_i (1 - G_ii), the hopping energy per site
 * (1/N) sum_{i != j} K_ij <c_i^dag c_j> (K of "Basics of DQMC" without mu),
 * and S(pi, pi) = (1/N) sum_ij (-1)^(x_i+y_i+x_j+y_j) <n_i n_j>.  Their Monte
 * Carlo averages over configurations are the measured observables.
 * batch may be any size (no workspace).  Errors: SLQ_ERR_ARG.
 */
int slq_measure_equal_time(slq_plan* plan, int32_t batch, const double* d_G, double* d_out, hipStream_t stream);

/*
 * slq_green_displaced - the time-displaced Green's function
 *   d_Gt[b] = G(tau_l, 0) = <c(tau_l) c^dag(0)> = B_l ... B_1 G,  l = slice,
 * 1 <= slice <= L, FP64 [batch][N][N] (G(beta, 0) = 1 - G): G from the
 * stabilised chain, then the slice products applied to it.  Those products
 * scale G's columns by up to exp(tau ||K + V||), so the result is accurate
 * while that factor stays far inside the FP64 range relative to G's entries
 * (beta of a few units at the workloads' couplings); a two-sided stabilised
 * form is not provided.  Uses the plan's workspace; FP64 products.
 * Errors: SLQ_ERR_ARG, SLQ_ERR_WORKSPACE, SLQ_ERR_DEVICE.
 */
int slq_green_displaced(slq_plan* plan, int32_t batch, const int8_t* d_s, int32_t slice, double* d_Gt,
                        int32_t* d_status, hipStream_t stream);

/*
 * Groups of independent chains of uneven size.  slq_group_create takes one
 * model per chain (N_c and L_c may all differ); chains with identical models
 * share an internal plan and are evaluated as one batch.  At creation the
 * tile shape of the FP64 chain GEMM is chosen for every distinct N by timing
 * the candidate shapes on the device (the choice then applies to every plan
 * of the process).  Synchronous; free with slq_group_destroy.
 * Errors: SLQ_ERR_ARG (a model fails the checks of slq_plan_create),
 * SLQ_ERR_DEVICE.
 */
typedef struct slq_group slq_group;
int slq_group_create(const slq_model* models, int32_t n_chains, slq_group** out);
/* As slq_group_create; flags SLQ_GROUP_EXACT_BATCHES: only chains with
 * identical models share a batch (no merging of lengths), which
 * slq_group_cumulative_step needs. */
enum { SLQ_GROUP_EXACT_BATCHES = 1 };
int slq_group_create_flags(const slq_model* models, int32_t n_chains, int32_t flags, slq_group** out);
int slq_group_destroy(slq_group* group);
/* Packed layouts (host arrays of n_chains + 1 entries): chain c's field is the
 * int8 [L_c][N_c] block at byte offset s_off[c] of d_s, its G the FP64
 * [N_c][N_c] block at element offset g_off[c] of d_G; the last entries are
 * the totals.  g_off may be NULL. */
int slq_group_layout(const slq_group* group, int64_t* s_off, int64_t* g_off);
/* JSON text describing the batches and the tuned tile shapes. */
int slq_group_describe(const slq_group* group, char* buf, size_t len);
/*
 * slq_group_weight / slq_group_green - Eq. 1's exact weight (and G) of every
 * chain: d_logabs, d_sign, d_status [n_chains], d_G packed as above.  The
 * batches are dealt to up to four streams of the group (largest estimated
 * work first, each to the least loaded stream); the whole evaluation (per
 * stream: gathers, the stabilised chains, QRs and final steps of its
 * batches, scatters) is recorded once, for a given set of pointers, as one
 * HIP graph whose parallel branches are the streams' parts, and replayed as
 * one graph launch afterwards (the first call with new pointers also runs it
 * eagerly).  The evaluation is ordered after prior work on `stream`, and
 * later work on `stream` waits for all of it.  Calls on one group must not
 * overlap in time.
 */
int slq_group_weight(slq_group* group, const int8_t* d_s, double* d_logabs, int8_t* d_sign,
                     int32_t* d_status, hipStream_t stream);
int slq_group_green(slq_group* group, const int8_t* d_s, double* d_G, double* d_logabs,
                    int8_t* d_sign, int32_t* d_status, hipStream_t stream);
/* Batches of the group: their number, and batch k's internal plan (owned by
 * the group; valid until slq_group_destroy), its chain count and, if
 * chain_ids is not NULL, the chain index of each batch position (host int32
 * [n_chains]).  The plan serves to create the batch's effective model
 * (slq_eff_create) and to fit it (slq_fit_effective on fields of that model). */
int slq_group_batches(const slq_group* group, int32_t* n_batches);
int slq_group_batch(slq_group* group, int32_t k, slq_plan** plan, int32_t* n_chains, int32_t* chain_ids);
/*
 * slq_group_cumulative_step - one cumulative update (steps (iii)-(iv) of
 * "Formalism of SLDQMC", Eq. 4) of every chain of the group, each with its
 * batch's effective model: effs[k] (created on batch k's plan) for batch k,
 * eff_sweeps sweeps of effective moves (eff_sweeps x its colour classes) per
 * proposal, judged by the exact FP64 weight of its own model.  In place on
 * the packed fields d_s and on d_logabs / d_sign [n_chains] (the current
 * weights); out (may be NULL): d_accepted int8, d_logA FP64, d_status int32
 * [n_chains].  Batch k's chains draw the random numbers of slq_cumulative_step
 * with chain0 = the number of chains in batches 0..k-1, batch position b as
 * chain chain0 + b.  The batches are dealt to the group's streams as for the
 * weight; the call is ordered after prior work on `stream`, and later work on
 * `stream` waits for all of it.  Errors: SLQ_ERR_ARG (a NULL effective model,
 * an effective model of another plan, a group that merged chains of
 * different lengths: create it with SLQ_GROUP_EXACT_BATCHES), SLQ_ERR_DEVICE.
 */
int slq_group_cumulative_step(slq_group* group, slq_eff* const* effs, int32_t eff_sweeps, uint64_t seed,
                              uint64_t step, int8_t* d_s, double* d_logabs, int8_t* d_sign,
                              int8_t* d_accepted, double* d_logA, int32_t* d_status, hipStream_t stream);

/*
 * slq_sweep_local - n_sweeps local-update DQMC sweeps ("Basics of DQMC") on
 * `batch` independent chains, in place.  For each slice l = 1..L and site
 * i = 0..N-1 in ascending order the flip s_{i,l} -> -s_{i,l} has ratio
 * R = 1 + delta (1 - G_ii), delta = exp(2 dtau xi s_{i,l}) - 1, with G the
 * Green's function whose cyclic chain ends at B_l; it is accepted iff
 * u < |R| (Metropolis on |W_f|) and G is updated by Sherman-Morrison
 * G -= (delta/R)(e_i - G[:,i]) G[i,:] (applied in delayed blocks).  After
 * each slice G <- B_l G B_l^{-1}; when l % n_stab == 0 G is recomputed and
 * the wrap drift max|G_wrapped - G_fresh| recorded.  The recomputation merges
 * the stabilised product B_l...B_1 (extended block by block as the sweep
 * moves up) with a stabilised B_L...B_{l+1} (built for every boundary when
 * the sweep starts), so a sweep costs O(L N^3) rather than O(L^2 N^3 / n_stab).
 * That stack of partial products lives in the plan's workspace, so the plan
 * must have been created with SLQ_PLAN_SWEEPS (else SLQ_ERR_WORKSPACE);
 * products are FP64 whatever the plan's chain precision.
 * u: key (seed, 1), counter (i, l-1, sweep0 + k, chain0 + b) for sweep k.
 * In/out: d_s [batch][L][N]; d_G [batch][N][N] must hold G of the incoming
 * fields (from slq_green) and holds G of the outgoing ones; d_logabs and
 * d_sign are advanced by log|R| and sign R of accepted flips.
 * Out: d_accepts int64 [batch] (accepted flips, summed over the sweeps),
 * d_drift FP64 [batch] (largest drift seen), d_status (may be NULL).
 */
int slq_sweep_local(slq_plan* plan, int32_t batch, int8_t* d_s, double* d_G,
                    double* d_logabs, int8_t* d_sign, int32_t n_sweeps,
                    uint64_t seed, uint64_t sweep0, uint64_t chain0,
                    int64_t* d_accepts, double* d_drift, int32_t* d_status,
                    hipStream_t stream);

/*
 * Effective bosonic action, Eq. 2 with symmetry-reduced couplings:
 *   S_eff(s) = c0 + sum_k lambda_k F_k(s),  F_k = 1/2 sum_x s_x h_k(x),
 *   h_k((i,l)) = sum over delta in spatial shell r_k of
 *                s_{i+delta, l+dl_k} + s_{i+delta, l-dl_k}   (dl_k > 0)
 *                s_{i+delta, l}                               (dl_k = 0)
 * with time taken modulo L.  Shell r holds the lattice offsets of the r-th
 * smallest squared length (0: (0,0); 1: (+-1,0),(0,+-1); 2: (+-1,+-1);
 * 3: (+-2,0),(0,+-2); 4: (+-2,+-1),(+-1,+-2); 5: (+-2,+-2)).
 * The term (r,dl) = (0,0) is the one-body term (a uniform field, the first
 * of the terms Eq. 2 leaves as "..."): h = 1 and F = sum_x s_x; a single
 * determinant has no s -> -s symmetry, so it is the leading term of ln|W_f|.
 * lambda_k = -beta J_k and c0 = -beta E_0, so S_eff approximates ln|W_f|
 * (Eq. 3).  A term needs 0 <= r <= 5, 0 <= dl <= L/2 and no site may be its
 * own partner.
 * Effective moves (step iii) act on colour classes: one class is one time
 * slice and one colour of the greedy colouring (ascending site index,
 * smallest free colour) of the graph of dl = 0 couplings; class index =
 * colour + n_colours*(l-1).  A move draws a class uniformly and applies
 * Metropolis u < exp(dS), dS = -2 s_x sum_k lambda_k h_k(x), to all its sites.
 * (slq_eff is declared with slq_plan above.)
 */

/* slq_eff_workspace_size - *bytes = device bytes of an effective model with
 * n_terms terms on `plan` (its tables, and room for an attached network's
 * parameters and move colouring).  Host only.
 * slq_eff_create - from host arrays terms [n_terms][2] = (r, dl),
 * lambda [n_terms], c0.  Builds the colour classes and copies the tables to
 * the device, into caller-owned device memory d_work (256-byte aligned, at
 * least the queried size) or, with d_work == NULL, into memory it allocates
 * once here and frees in slq_eff_destroy.  No later call on the model
 * allocates.  Synchronous.  Errors: SLQ_ERR_ARG, SLQ_ERR_WORKSPACE
 * (work_bytes too small), SLQ_ERR_DEVICE. */
int slq_eff_workspace_size(const slq_plan* plan, int32_t n_terms, size_t* bytes);
int slq_eff_create(slq_plan* plan, int32_t n_terms, const int32_t* terms,
                   const double* lambda, double c0, void* d_work, size_t work_bytes, slq_eff** out);
int slq_eff_destroy(slq_eff* eff);
/* Number of colour classes (n_colours * L). */
int slq_eff_classes(const slq_eff* eff, int32_t* n_classes);
/* Replace (c0, lambda) from device memory d_theta [1 + n_terms] on `stream`
 * (e.g. the output of slq_fit_effective). */
int slq_eff_set_theta(slq_eff* eff, const double* d_theta, hipStream_t stream);

/*
 * slq_eff_sweep - n_moves effective moves on each of `batch` fields, in place
 * (step iii of the paper, "Formalism of SLDQMC").  The class of move m of
 * chain b uses counter (0, m, step, chain0+b); the Metropolis draw of site
 * (i, l) uses counter (1 + (l-1)*N + i, m, step, chain0+b); key (seed, 2).
 * Out (may be NULL): d_accepts int64 [batch], d_dS FP64 [batch] = sum of the
 * accepted dS.
 */
int slq_eff_sweep(slq_plan* plan, const slq_eff* eff, int32_t batch, int8_t* d_s,
                  int32_t n_moves, uint64_t seed, uint64_t step, uint64_t chain0,
                  int64_t* d_accepts, double* d_dS, hipStream_t stream);

/* slq_eff_features - d_F FP64 [batch][n_terms] = F_k(s_b) (exact half-integers). */
int slq_eff_features(slq_plan* plan, const slq_eff* eff, int32_t batch,
                     const int8_t* d_s, double* d_F, hipStream_t stream);

/*
 * Learned effective action (the "..." of Eq. 2: interactions beyond the pair
 * couplings).  A small convolutional network on the field viewed as
 * [L][ly][lx], periodic in all three axes:
 *   a1[c] = b1[c] + sum_k W1[c][k] s(x + o(k)),         h1 = tanh(a1),  c = 0..7
 *   a2[c] = b2[c] + sum_{c',k} W2[c][c'][k] h1[c'](x + o(k)),  h2 = tanh(a2)
 *   S_net = b3 + sum_c w3[c] sum_x h2[c](x)
 * with k = 0..26 and o(k) = (k/9 - 1, (k/3)%3 - 1, k%3 - 1) along (time, y, x).
 * Parameters: SLQ_NET_PARAMS FP64 values W1[8][27], b1[8], W2[8][8][27],
 * b2[8], w3[8], b3 (caller-owned device memory).  The learned action is
 * S_theta = S_lin + S_net; arithmetic in FP32 (net_prec = SLQ_PREC_FP32) or
 * FP64.  All reductions have a fixed order (deterministic results).
 */
#define SLQ_NET_PARAMS 1969

/* The network calls below need a plan created with SLQ_PLAN_NET (else
 * SLQ_ERR_WORKSPACE). */
/* d_S[b] = S_net(s_b). */
int slq_net_forward(slq_plan* plan, int32_t net_prec, int32_t batch, const int8_t* d_s,
                    const double* d_params, double* d_S, hipStream_t stream);
/* Gradient of the loss (1/B) sum_b (S_net(s_b) - r_b)^2, r_b = d_y[b] - S_lin(s_b),
 * S_lin from the linear model of `eff` (its current c0 and lambda): the network
 * is trained on the residual of the linear fit.  d_grad [SLQ_NET_PARAMS];
 * d_loss [1] (may be NULL).  1 <= batch <= max_batch. */
int slq_net_gradient(slq_plan* plan, const slq_eff* eff, int32_t net_prec, int32_t batch,
                     const int8_t* d_s, const double* d_y, const double* d_params,
                     double* d_grad, double* d_loss, hipStream_t stream);
/* One Adam step (Kingma & Ba, with bias correction) of n parameters; t >= 1. */
int slq_net_adam(int32_t n, double* d_params, const double* d_grad, double* d_m, double* d_v,
                 int64_t t, double lr, double beta1, double beta2, double eps, hipStream_t stream);
/*
 * slq_eff_set_net - attach a copy of the network parameters d_params to `eff`
 * (or detach with d_params = NULL: the linear model is the fallback).  While
 * attached, slq_eff_sweep and slq_cumulative_step use S_lin + S_net: the move
 * classes are one slice and one colour of the greedy colouring of the dl = 0
 * couplings together with all pairs within spatial Chebyshev distance 4 (a
 * flip changes h2 within distance 2, so the neighbourhoods touched by the
 * sites of a class are disjoint), one class drawn uniformly per move as
 * before; Eq. 4 uses S_net(s') - S_net(s) from full forward passes.  Needs
 * lx, ly, L >= 5.  The colouring is built on the first attach (synchronous).
 * net_prec must be SLQ_PREC_FP64 (else SLQ_ERR_ARG): the moves keep the
 * network's activations up to date incrementally, and only in FP64 does a
 * move and its reverse change the action by negatives up to round-off, which
 * Eq. 4's acceptance needs to stay exact.  Training and the forward and
 * gradient calls above may run in FP32.
 */
int slq_eff_set_net(slq_eff* eff, const double* d_params, int32_t net_prec, hipStream_t stream);
/* Number of move classes while a network is attached. */
int slq_eff_net_classes(const slq_eff* eff, int32_t* n_classes);

/*
 * slq_cumulative_step - one cumulative update (steps iii-iv, Eq. 4) of each
 * of `batch` chains: s' = s after n_moves effective moves (as slq_eff_sweep
 * with the same seed/step/chain0), logA = [ln|W(s')| - ln|W(s)|] -
 * [S_eff(s') - S_eff(s)], accepted iff ln u < min(0, logA) with u from key
 * (seed, 3), counter (0, 0, step, chain0+b).  On acceptance s, logabs and
 * sign are replaced by those of s'.  d_logabs / d_sign must hold the exact
 * weight of the incoming fields (from slq_weight).
 * Out (may be NULL): d_accepted int8 [batch], d_logA FP64 [batch], d_status.
 */
int slq_cumulative_step(slq_plan* plan, const slq_eff* eff, int32_t batch,
                        int8_t* d_s, double* d_logabs, int8_t* d_sign,
                        int32_t n_moves, uint64_t seed, uint64_t step, uint64_t chain0,
                        int8_t* d_accepted, double* d_logA, int32_t* d_status,
                        hipStream_t stream);

/*
 * slq_fit_effective - multi-linear regression of Eq. 3 (step ii):
 * ordinary least squares with an intercept of y_n = d_logabs[n] on the
 * features F_k(s_n) of the terms of `eff`, for n_samples fields d_S
 * [n_samples][L][N].  Writes d_theta [1 + n_terms] = (c0, lambda_1..K) and
 * d_r2 [1] = 1 - sum (y - yhat)^2 / sum (y - ybar)^2 (the paper's R^2 score,
 * "Results").  Needs n_samples >= n_terms + 2.  A singular system leaves
 * d_theta as NaN.  Device work only; does not change `eff`.  Any n_samples:
 * the features are computed max_batch fields at a time into the plan's
 * buffers (two passes: sums, then the residuals of R^2), so nothing is
 * allocated.
 */
int slq_fit_effective(slq_plan* plan, const slq_eff* eff, int64_t n_samples,
                      const int8_t* d_S, const double* d_logabs,
                      double* d_theta, double* d_r2, hipStream_t stream);

/*
 * The paper's own workload ("Results", Eq. 6): spin-1/2 fermions on a bilayer
 * (intralayer hopping t, chemical potential mu of the plan's model) coupled
 * by H_sf = -xi sum_i s^z_i (sigma^z_{i1} - sigma^z_{i2}) to transverse-field
 * Ising spins H_s = -J sum_<ij> s^z s^z - h sum_i s^x.  The field s_{i,l}
 * (int8 [batch][L][N], one spin per site of the layer pair and slice) has the
 * sign-free weight
 *   omega(s) = phi(s) [W_f(s) W_f(-s)]^2,
 * W_f the single-flavour determinant of this header (two of the four flavours
 * see xi s, two -xi s), and phi the weight of the Ising spins alone (the
 * factor of Eq. 1 without fermions), from the quantum-to-classical mapping of H_s:
 *   ln phi = dtau J sum_l sum_<ij> s_{i,l} s_{j,l} + K_tau sum_{i,l} s_{i,l} s_{i,l+1},
 *   K_tau = -1/2 ln tanh(dtau h)   (up to a constant; bonds as in K).
 * Every call evaluates 2 batch fields [s ; -s], so the plan's max_batch must
 * be >= 2 batch (else SLQ_ERR_WORKSPACE); FP64 chains only; h > 0;
 * lx, ly, L >= 2.
 */
typedef struct slq_bilayer {
  double J;  /* ferromagnetic Ising coupling */
  double h;  /* transverse field, > 0 */
} slq_bilayer;

/* d_logw[b] = ln omega(s_b) (-inf when a determinant vanishes). */
int slq_bilayer_weight(slq_plan* plan, const slq_bilayer* bl, int32_t batch, const int8_t* d_s,
                       double* d_logw, int32_t* d_status, hipStream_t stream);
/* As slq_bilayer_weight, and d_G FP64 [2 batch][N][N]: G of s_b at b and of
 * -s_b at batch + b (the chain B_L ... B_1). */
int slq_bilayer_green(slq_plan* plan, const slq_bilayer* bl, int32_t batch, const int8_t* d_s, double* d_G,
                      double* d_logw, int32_t* d_status, hipStream_t stream);
/*
 * slq_bilayer_sweep_local - local-update sweeps of the bilayer weight
 * ("Basics of DQMC") in place: sites ascending within slices 1..L; the flip
 * of s_{i,l} has ratio phi'/phi (R_a R_b)^2, R_a = 1 + delta_a (1 - G_a,ii),
 * delta_a = exp(2 dtau xi s_{i,l}) - 1 from the G of s, R_b likewise from the
 * G of -s with delta_b = exp(-2 dtau xi s_{i,l}) - 1; accepted iff u < ratio,
 * u from key (seed, 1), counter (i, l-1, sweep0 + k, chain0 + b); both
 * Green's functions then take their Sherman-Morrison update (undelayed),
 * are wrapped after each slice and recomputed from the cyclic chain every
 * n_stab slices, recording the drift.
 * d_G [2 batch][N][N] holds the incoming Green's functions (slq_bilayer_green)
 * and the outgoing ones; d_logw is advanced by ln ratio of accepted flips.
 * Out (may be NULL): d_accepts int64 [batch], d_drift FP64 [batch], d_status.
 */
int slq_bilayer_sweep_local(slq_plan* plan, const slq_bilayer* bl, int32_t batch, int8_t* d_s, double* d_G,
                            double* d_logw, int32_t n_sweeps, uint64_t seed, uint64_t sweep0, uint64_t chain0,
                            int64_t* d_accepts, double* d_drift, int32_t* d_status, hipStream_t stream);
/*
 * slq_bilayer_cumulative_step - one cumulative update (Eq. 4) of each chain
 * with the bilayer weight as the judge: effective moves as slq_eff_sweep
 * (same counters as slq_cumulative_step), logA = [ln omega(s') - ln omega(s)]
 * - [S_eff(s') - S_eff(s)], accepted iff ln u < min(0, logA) (u from key
 * (seed, 3), counter (0, 0, step, chain0 + b)); on acceptance s and d_logw
 * are replaced.  d_logw must hold ln omega of the incoming fields.
 * Out (may be NULL): d_accepted int8 [batch], d_logA FP64 [batch], d_status.
 */
int slq_bilayer_cumulative_step(slq_plan* plan, const slq_eff* eff, const slq_bilayer* bl, int32_t batch,
                                int8_t* d_s, double* d_logw, int32_t n_moves, uint64_t seed, uint64_t step,
                                uint64_t chain0, int8_t* d_accepted, double* d_logA, int32_t* d_status,
                                hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* SLQ_H */
