// Internal declarations of libslq: the plan, the effective-model handle,
// device helpers (Philox4x64-10, wavefront reductions) and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/slq.h"

namespace slq {

void set_error(const std::string& msg);

#define SLQ_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ::slq::set_error(std::string(#call) + ": " + hipGetErrorString(e_));         \
      return SLQ_ERR_DEVICE;                                                       \
    }                                                                              \
  } while (0)

#define SLQ_LAUNCHED()                                                             \
  do {                                                                             \
    hipError_t e_ = hipGetLastError();                                             \
    if (e_ != hipSuccess) {                                                        \
      ::slq::set_error(std::string("kernel launch: ") + hipGetErrorString(e_));    \
      return SLQ_ERR_DEVICE;                                                       \
    }                                                                              \
  } while (0)

// Return the status of a library call from the enclosing function unless OK.
#define SLQ_TRY(x)                 \
  do {                             \
    int rc_ = (x);                 \
    if (rc_ != SLQ_OK) return rc_; \
  } while (0)

// Raise a kernel's dynamic-LDS limit to the 160 KiB of a gfx950 CU, once per
// kernel and process (so no attribute call happens while a graph is recorded).
inline void allow_max_lds(const void* fn) {
  static std::mutex mu;
  static std::vector<const void*> done;
  std::lock_guard<std::mutex> lk(mu);
  for (const void* f : done)
    if (f == fn) return;
  hipFuncAttributes attr;
  if (hipFuncGetAttributes(&attr, fn) == hipSuccess)
    hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - (int)attr.sharedSizeBytes);
  (void)hipGetLastError();  // a refused attribute must not surface as the next launch's error
  done.push_back(fn);
}

// ---------------------------------------------------------------- Philox ----
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 64x64
// multiplies with the Weyl-sequence key schedule.
struct u64x4 {
  uint64_t v[4];
};

__device__ __forceinline__ u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  u64x4 o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

__device__ __forceinline__ double philox_uniform(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                 uint64_t k0, uint64_t k1) {
  return (double)(philox4x64_10(c0, c1, c2, c3, k0, k1).v[0] >> 11) * 0x1.0p-53;
}

__device__ __forceinline__ uint32_t philox_below(uint32_t n, uint64_t c0, uint64_t c1, uint64_t c2,
                                                 uint64_t c3, uint64_t k0, uint64_t k1) {
  const uint64_t w = philox4x64_10(c0, c1, c2, c3, k0, k1).v[0] >> 32;
  return (uint32_t)((w * (uint64_t)n) >> 32);
}

enum : uint64_t { TAG_LOCAL = 1, TAG_EFFECTIVE = 2, TAG_CUMULATIVE = 3 };

// Workgroup barrier that orders LDS traffic only: each wave's LDS accesses
// complete before it, but its global loads stay in flight (a full
// __syncthreads() also waits for every outstanding global access).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ------------------------------------------------------------ reductions ----
// Whole-wave reductions (every lane active) with DPP lane moves inside rows of
// 16 lanes (quad permutations, row rotations) and lane reads for the four row
// results: no LDS round trips.  Every lane returns the same value, combined in
// a fixed order.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double read_lane(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}
enum : int { DPP_QUAD_XOR1 = 0xB1, DPP_QUAD_XOR2 = 0x4E, DPP_ROW_ROR4 = 0x124, DPP_ROW_ROR8 = 0x128 };
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<DPP_QUAD_XOR1>(v);
  v += dpp_move<DPP_QUAD_XOR2>(v);
  v += dpp_move<DPP_ROW_ROR4>(v);
  v += dpp_move<DPP_ROW_ROR8>(v);
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}
template <int CTRL>
__device__ __forceinline__ int dpp_move_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
// Largest v over the wave, ties to the smallest index i (exact: any order of
// combination gives the same pair).
__device__ __forceinline__ void argmax_merge(double& v, int& i, double ov, int oi) {
  if (ov > v || (ov == v && oi < i)) {
    v = ov;
    i = oi;
  }
}
template <int CTRL>
__device__ __forceinline__ void argmax_step(double& v, int& i) {
  const double ov = dpp_move<CTRL>(v);
  const int oi = dpp_move_i32<CTRL>(i);
  argmax_merge(v, i, ov, oi);
}
__device__ __forceinline__ void wave_argmax(double& v, int& i) {
  argmax_step<DPP_QUAD_XOR1>(v, i);
  argmax_step<DPP_QUAD_XOR2>(v, i);
  argmax_step<DPP_ROW_ROR4>(v, i);
  argmax_step<DPP_ROW_ROR8>(v, i);
  double bv = read_lane(v, 0);
  int bi = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
  for (int r = 16; r < 64; r += 16) argmax_merge(bv, bi, read_lane(v, r), __builtin_amdgcn_readlane(i, r));
  v = bv;
  i = bi;
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_move<DPP_QUAD_XOR1>(v));
  v = fmax(v, dpp_move<DPP_QUAD_XOR2>(v));
  v = fmax(v, dpp_move<DPP_ROW_ROR4>(v));
  v = fmax(v, dpp_move<DPP_ROW_ROR8>(v));
  return fmax(fmax(read_lane(v, 0), read_lane(v, 16)), fmax(read_lane(v, 32), read_lane(v, 48)));
}
// Larger of a and b, NaN if either is NaN (fmax returns the other operand and
// would hide a non-finite value from a max-reduction).
__device__ __forceinline__ double nan_max(double a, double b) {
  if (a != a) return a;
  if (b != b) return b;
  return a > b ? a : b;
}
// wave_max that propagates NaN: any lane's NaN reaches every lane.
__device__ __forceinline__ double wave_max_nan(double v) {
  v = nan_max(v, dpp_move<DPP_QUAD_XOR1>(v));
  v = nan_max(v, dpp_move<DPP_QUAD_XOR2>(v));
  v = nan_max(v, dpp_move<DPP_ROW_ROR4>(v));
  v = nan_max(v, dpp_move<DPP_ROW_ROR8>(v));
  return nan_max(nan_max(read_lane(v, 0), read_lane(v, 16)), nan_max(read_lane(v, 32), read_lane(v, 48)));
}

// ------------------------------------------------------------------ plan ----
struct Plan {
  slq_model m;
  int n;          // sites N
  int L;          // slices
  int max_batch;
  int device;
  size_t bytes;
  double* base;   // single allocation holding everything below
  double* E;      // [N][N] exp(-dtau K)
  double* Einv;   // [N][N] exp(+dtau K)
  double* consts; // [0] exp(-dtau xi), [1] exp(+dtau xi), [2] exp(dtau mu), [3] exp(-dtau mu)
  double* tabs;   // 1-D propagator tables, 4*(lx+ly)
  float* E32;     // [N][N] E in FP32 (reduced-precision chains)
  void* E16;      // [N][N] bf16(E32)
  // per-item N x N buffers
  double *Xa, *Xb, *W, *U, *V, *Vt;
  // per-item vectors
  double *D, *invD, *Tblk;  // D, 1/D: [N]; compact-WY T blocks: (N + 32) * 32 per field
  int32_t* perm;            // [N]
  double* xnorm2;           // [N]: squared column norms of a structured block product
  int32_t* nref;            // [max_batch] reflectors with tau != 0 in the latest QR
  int32_t* status;          // [max_batch] scratch status when caller passes NULL
  int32_t *nref2, *status2; // [max_batch] each: reflector count and status of the QR of M (det_qr.hip)
  int8_t* s_work;           // [max_batch][L][N] proposal fields
  double* dvec;             // [max_batch] scratch doubles
  double* dvec2;            // [max_batch] scratch doubles
  int64_t* ivec;            // [max_batch] scratch counters
  // local sweeps: delayed-update vectors per item
  double *dX, *dY;          // [N][KD] and [KD][N]
  double* dA;               // [KD]
  // cumulative updates
  double *F_old, *F_new;    // [max_batch][64] effective-action features
  int8_t* sgn_work;         // [max_batch]
  int8_t* sgn_work2;        // [max_batch]
  // optional event timing of the chain-product GEMM launches
  // parts: SLQ_PROFILE_CHAIN, SLQ_PROFILE_STAB, SLQ_PROFILE_FINISH
  bool prof = false;
  std::vector<hipEvent_t> ev[3];  // start/stop pairs per part
  size_t ev_used[3] = {0, 0, 0};
  double prof_flops[3] = {0.0, 0.0, 0.0};
  // learned-action buffers (SLQ_PLAN_NET): device region in the workspace and
  // the host-side view of it
  void* net_base = nullptr;
  void* net_state = nullptr;
  // the workspace was allocated by slq_plan_create (d_work NULL) and is freed with the plan
  bool owns_base = false;
  // accumulators of the chunked regression (FIT_ACC_DOUBLES)
  double* fit_acc = nullptr;
  // tile configuration of the FP64 chain GEMM chosen by the autotuner (-1: default)
  int gemm_cfg = -1;
  // structured (Kronecker) slice products: register line length (0: lattice
  // too large, dense products), coefficient windows [E x | E y | E^-1 x | E^-1 y]
  // of 2P entries each, and the vectors per workgroup (0: default)
  int kron_P = 0;
  double* kron_w = nullptr;
  int kron_nb = 0;
  // checkerboard split of the kinetic factor (SLQ_PREC_CHECKERBOARD): E and
  // E^{-1} hold E_cb and its inverse, and the structured products apply it
  // bond group by bond group (kron_nb is then its vectors per workgroup)
  bool cb = false;
  // [max_batch] or null: the first stabilisation block of each field's chain
  // (earlier blocks leave U D V = I 1 I; set by groups that batch chains of
  // several lengths, structured products only; device memory the plan does not own)
  const int32_t* first_block = nullptr;
  // blocked QR workspace: outer compact-WY factors, Gram blocks, V^T A products
  double* qrws = nullptr;

  // stabilised partial products kept by local sweeps (SLQ_PLAN_SWEEPS) for
  // stack_batch = max_batch fields (see sweep_stacked)
  double* stack = nullptr;
  int stack_batch = 0;
};

// Slice products through launch_kron are available (circulant lines or
// checkerboard bonds) / are the chain's own products.
inline bool has_structured(const Plan& p) { return p.cb || p.kron_P > 0; }
inline bool structured_chain(const Plan& p) { return p.cb || (p.m.chain_prec == SLQ_PREC_FP64 && p.kron_P > 0); }

struct Eff {
  Plan* plan;
  int n_terms;
  int n_colours;
  int n_classes;
  int32_t* d_terms;      // [n_terms][2]
  double* d_theta;       // [1 + n_terms] (c0, lambda)
  int32_t* d_col_sites;  // sites sorted by colour
  int32_t* d_col_off;    // [n_colours + 1]
  int max_class;         // largest colour class
  int32_t* d_shell_off;  // shell offset table [6 + 1]
  int32_t* d_shell_dxy;  // [total][2]
  std::vector<int32_t> h_terms;  // host copy of the terms
  void* base = nullptr;           // device tables (caller-owned unless owns_base)
  bool owns_base = false;
  // learned action (optional)
  bool net_on = false;
  int net_prec = 0;
  double* d_net = nullptr;          // [1969] parameters (owned copy)
  int32_t* d_ncol_sites = nullptr;  // colouring that also separates the network's range
  int32_t* d_ncol_off = nullptr;
  int n_ncolours = 0;
  // every partner relation of the two-body terms, one entry per (offset, +-dl):
  // u | (dt + 2048) << 8 | k << 20, u the index of the spatial offset in d_uoff
  int n_pairs = 0;
  int32_t* d_pairs = nullptr;
  int n_uoff = 0;
  int32_t* d_uoff = nullptr;  // [n_uoff][2] the distinct spatial offsets (dx, dy) of the pairs
};

// Device view of an effective model.
struct EffDev {
  int lx, ly, L, N;
  int n_terms, n_colours, n_classes;
  const int32_t* terms;      // [K][2]
  const double* theta;       // [1 + K]
  const int32_t* col_sites;  // [N]
  const int32_t* col_off;    // [n_colours + 1]
  const int32_t* shell_off;  // [7]
  const int32_t* shell_dxy;  // [25][2]
  int n_pairs;
  const int32_t* pairs;      // [n_pairs], see Eff
  int n_uoff;
  const int32_t* uoff;       // [n_uoff][2]
};
EffDev eff_dev_view(const Plan& p, const Eff& e);

// h_k((i, l)) of term k at site i, slice l (0-based) of one field s [L][N];
// 1 for the one-body term (0, 0)
__device__ __forceinline__ int local_field_dev(const EffDev& d, const int8_t* __restrict__ s, int k, int i, int l) {
  const int r = d.terms[2 * k], dl = d.terms[2 * k + 1];
  if (r == 0 && dl == 0) return 1;
  const int x = i % d.lx, y = i / d.lx;
  int h = 0;
  const int lp = (l + dl) % d.L, lm = (l - dl + d.L) % d.L;
  for (int o = d.shell_off[r]; o < d.shell_off[r + 1]; ++o) {
    const int xx = ((x + d.shell_dxy[2 * o]) % d.lx + d.lx) % d.lx;
    const int yy = ((y + d.shell_dxy[2 * o + 1]) % d.ly + d.ly) % d.ly;
    const int j = xx + d.lx * yy;
    if (dl == 0) {
      h += s[(long)l * d.N + j];
    } else {
      h += s[(long)lp * d.N + j] + s[(long)lm * d.N + j];
    }
  }
  return h;
}

constexpr int MAX_TERMS_ABI = 64;  // terms of an effective model
constexpr int QR_NB = 16;     // Householder / LU panel width
constexpr int QR_NBO = 128;   // outer block of the blocked QR
long qr_workspace_per_field(int N);  // doubles per field of Plan::qrws
constexpr int SWEEP_KD = 32;  // delayed local updates per flush

// ------------------------------------------------------------- launchers ----
int launch_kinetic(Plan& p, hipStream_t st);

// C[b] = alpha * rowscale[b] o (op(A[b]) * diag(r_b) * op(B[b])) + beta * C[b]
struct GemmArgs {
  int M, N, K;
  const double* A;
  long lda, strideA;
  const double* B;
  long ldb, strideB;
  double* C;
  long ldc, strideC;
  const int8_t* S;    // field: r_b[k] = consts[s > 0 ? 0 : 1] ^ (+1 or -1); null = no scaling
  long strideS;
  int slice;          // 0-based slice of S used for the scaling
  int inv_scale;      // 0: r = exp(-dtau xi s), 1: r = exp(+dtau xi s)
  const double* consts;
  const double* rowscale;  // null = none
  long strideRS;
  double alpha, beta;
  int a_upper;        // A is upper triangular: entries with k < m are taken as zero
  const int32_t* brow = nullptr;  // a_upper only: row k of op(B) is row brow[k] of B ([batch] + strideBrow)
  long strideBrow = 0;
  int s_out;          // apply the field factor to the rows of C instead of the rows of op(B)
  int c_ident = 0;      // beta != 0: C is read as the identity (its own diagonal), not from memory
  int c_zero_rows = 0;  // beta != 0: rows m < c_zero_rows of C are read as zero, not from memory
  int cfg = -1;       // tile configuration (GemmCfg), -1 = default choice
  int batch;
};
int launch_gemm(const GemmArgs& a, bool transA, bool transB, hipStream_t st);
// Tile configurations (TM x TN, K stage depth) of the FP64 GEMM.
enum GemmCfg {
  GEMM_16 = 0,     // 16 x 16, 1 wavefront
  GEMM_32x64,      // 32 x 64, 4 wavefronts (thin panels)
  GEMM_128,        // 128 x 128, K 8
  GEMM_96,         // 96 x 96, K 8
  GEMM_80_K4,      // 80 x 80, 5 wavefronts, K 4
  GEMM_80_K8,      // 80 x 80, 5 wavefronts, K 8
  GEMM_160x80,     // 160 x 80, 10 wavefronts, K 8
  GEMM_64,         // 64 x 64, K 8
  GEMM_48,         // 48 x 48, 3 wavefronts, K 8
  GEMM_64x128,     // 64 x 128, 8 wavefronts, K 8
  GEMM_128x64,     // 128 x 64, 8 wavefronts, K 8 (products of the blocked QR)
  GEMM_16x64,      // 16 x 64, 4 wavefronts, K 16 (16-row products)
  GEMM_128x16,     // 128 x 16, 4 wavefronts, K 8 (16-column edges)
  GEMM_32x64_K32,  // 32 x 64, 4 wavefronts, K 32 (thin products with long K)
  GEMM_16x64_K32,  // 16 x 64, 4 wavefronts, K 32
  GEMM_BIG,        // 128 x 128, 4 wavefronts of 64 x 64, K 16 (tile-aligned, else 128 x 64)
  GEMM_LEAN,       // 128 x 64, 8 wavefronts, K 8, no bounds checks (tile-aligned, else 128 x 64)
  GEMM_NCFG
};
int launch_gemm_cfg(const GemmArgs& a, bool transA, bool transB, int cfg, hipStream_t st);
// GEMM_BIG: whether the large-tile kernel takes the product (shape multiple of its
// tiles, aligned operands, no transposed B, no field scaling), and its launch
bool gemm_big_ok(const GemmArgs& a, bool transA, bool transB);
int launch_gemm_big(const GemmArgs& a, bool transA, hipStream_t st);
// GEMM_LEAN: 128 x 64 tiles without bounds checks (untransposed, tile-aligned, aligned operands)
bool gemm_lean_ok(const GemmArgs& a, bool transA, bool transB);
int launch_gemm_lean(const GemmArgs& a, hipStream_t st);
int default_gemm(int M, int N);
struct Plan;
int tune_chain_gemm(Plan& p, int batch, hipStream_t st, float* best_ms);

// Reduced-precision chain GEMM: C(f32)[b] = A(f32, shared) diag(d_slice) B[b] (f32 or f64)
struct LpArgs {
  int M, N, K;
  const float* A;
  long lda;
  const void* B;
  long ldb, strideB;
  float* C;
  long ldc, strideC;
  const int8_t* S;
  long strideS;
  int slice;
  const double* consts;
  int batch;
};
int launch_gemm_lp(const LpArgs& a, int prec, bool b_is_f64, hipStream_t st);
int launch_first_slice_f32(Plan& p, int batch, const int8_t* s, long strideS, int slice, float* X, hipStream_t st);
int launch_widen(const float* a, double* b, long n, hipStream_t st);
int launch_narrow(const double* a, float* b, long n, hipStream_t st);
// BF16 chain with k-contiguous operands (N % 8 == 0), see gemm_lp.hip
struct LpTArgs;
int launch_bf16t_product(Plan& p, int batch, const void* BT, void* out, int out_f64, const int8_t* s, long strideS,
                         int slice_next, hipStream_t st);
int launch_f32t_product(Plan& p, int batch, const void* BT, void* out, int out_f64, const int8_t* s, long strideS,
                        int slice_next, hipStream_t st);
int launch_bt_prepare(int N, int batch, const double* X, long strideX, const int8_t* S, long strideS, int slice,
                      const double* consts, void* BT, int prec, hipStream_t st);
int launch_to_bf16(const float* a, void* b, long n, hipStream_t st);

// Structured slice products X <- B X for a block of slices (see kron.hip).
struct KronArgs {
  const double* in;  // [batch] N x N (stride strideIn); null: start from the identity
  long strideIn;
  double* out;       // may equal in
  long strideOut;
  int rows;          // 0: the operator acts on the columns, 1: on the rows (X <- X B^T)
  const int8_t* s;   // fields [batch][L][N]
  int slice0, count, step;  // slices (slice0 + k step) mod L, k = 0..count-1, first applied first
  int scale;         // 0: E only, 1: E diag(d_l) (B_l), 2: diag(d_l) E (B_l^T)
  int inv;           // E^{-1} and 1/d_l instead
  int nb = 0;        // vectors per workgroup (0: the plan's choice)
  int batch;
  double* norm2 = nullptr;  // rows == 0: [batch][N] squared 2-norms of the output columns, or null
  const int32_t* first_block = nullptr;  // [batch] or null: block < first_block[b] leaves field b's X as it is
  int block = 0;                         // stabilisation block of the launch (first_block only)
};
int kron_line_size(int lx, int ly);
// Workgroup-to-block order, XCD-aware: the hardware deals workgroups to the
// 8 XCDs in turn, so hardware ids g, g + 8, ..., g + 8 (G - 1) run side by
// side on one XCD; they take the G consecutive vector blocks G p .. G p + G - 1,
// which share the 128-byte lines of the field's rows (nb vectors of 8 bytes
// per row and block: G = 128 / (8 nb), at least 2), so each line is fetched
// into one L2 only.  A permutation within each aligned group of 8 G ids (the
// grid is rounded up to a multiple of 8 G).
__host__ __device__ inline int kron_group(int nb) { return nb >= 8 ? 2 : 16 / nb; }
__device__ __forceinline__ int kron_item(int g, int G) {
  return (g & ~(8 * G - 1)) | ((g & 7) * G) | ((g >> 3) & (G - 1));
}
// Checkerboard products (SLQ_PREC_CHECKERBOARD): launch_kron hands them to
// launch_cb, which takes the same arguments.
int launch_cb(Plan& p, const KronArgs& a, hipStream_t st);
int launch_cb_dense(Plan& p, hipStream_t st);
bool cb_width_ok(const Plan& p, int nb);
int cb_default_nb(const Plan& p);
int kron_default_nb(const Plan& p);
bool kron_width_ok(const Plan& p, int nb);
int launch_kron_windows(Plan& p, hipStream_t st);
int launch_kron(Plan& p, const KronArgs& a, hipStream_t st);
int tune_kron(Plan& p, int batch, hipStream_t st, float* best_ms);

// Chain helpers
int launch_first_slice(Plan& p, int batch, const int8_t* s, long strideS, int slice, double* X, hipStream_t st);
int launch_set_identity(Plan& p, int batch, double* X, hipStream_t st);
// A stabilised factorisation U D V of [batch] fields, N x N / N / N x N per
// field packed densely, plus the Householder count whose parity is det U.
struct UdvRef {
  double* U;
  double* D;
  double* V;
  int32_t* nref;
};
inline UdvRef plan_udv(Plan& p) { return UdvRef{p.U, p.D, p.V, p.nref}; }

// QR of X diag(o.D) with column pre-pivoting.  Reads o.D, then overwrites it
// with |diag R|; writes Q to o.U, the reflection count to o.nref, R above the
// diagonal to W, and invD, perm.  launch_qr keeps one workgroup per field for
// the whole factorisation (small N); launch_qr_blocked factors panels in LDS
// and updates with MFMA GEMMs (it uses Xa or Xb, whichever does not hold X,
// and Vt, dX, dY as scratch).
int launch_qr(Plan& p, int batch, const double* X, const UdvRef& o, int32_t* status, hipStream_t st);
// norm2 (optional): squared 2-norms of the columns of X, [batch][N]
// form_q = false leaves o.U untouched (R, |diag R|, the permutation and the
// reflector count only).
int launch_qr_blocked(Plan& p, int batch, const double* X, const UdvRef& o, int32_t* status, hipStream_t st,
                      const double* norm2 = nullptr, bool form_q = true);
inline int launch_qr(Plan& p, int batch, const double* X, int32_t* status, hipStream_t st) {
  return launch_qr(p, batch, X, plan_udv(p), status, st);
}
inline int launch_qr_blocked(Plan& p, int batch, const double* X, int32_t* status, hipStream_t st,
                             const double* norm2 = nullptr) {
  return launch_qr_blocked(p, batch, X, plan_udv(p), status, st, norm2);
}
// V <- diag(1/D) triu(R) Pi^T, the V update of a block whose V_prev is the
// identity (R in p.W, 1/D in p.invD, Pi in p.perm)
int launch_first_v(Plan& p, int batch, double* V, hipStream_t st);
// V_out <- diag(1/D) triu(R) Pi^T V_in (V_out != V_in)
int launch_v_update(Plan& p, int batch, const double* V_in, double* V_out, hipStream_t st);
// log|det(1 + U D V)|, its sign and optionally G = (1 + U D V)^{-1}; W is
// scratch.
int launch_finish(Plan& p, int batch, const UdvRef& f, double* G, double* logabs, int8_t* sign, int32_t* status,
                  hipStream_t st);
int launch_finish_lu(Plan& p, int batch, const UdvRef& f, double* G, double* logabs, int8_t* sign, int32_t* status,
                     hipStream_t st);
inline int launch_finish(Plan& p, int batch, double* G, double* logabs, int8_t* sign, int32_t* status,
                         hipStream_t st) {
  return launch_finish(p, batch, plan_udv(p), G, logabs, sign, status, st);
}
int launch_check_spins(Plan& p, int batch, const int8_t* s, int32_t* status, hipStream_t st);
// log|det(1 + U D V)| and sign from an R-only blocked QR of M (no G); uses Xa,
// Xb, W, Vt, perm, invD, qrws, nref2, status2.  use_det_qr: N > 64 and f
// lies outside those buffers.
bool use_det_qr(const Plan& p, const UdvRef& f);
int launch_det_qr(Plan& p, int batch, const UdvRef& f, double* logabs, int8_t* sign, int32_t* status,
                  hipStream_t st);

int run_chain(Plan& p, int batch, const int8_t* s, int slice0, int32_t* status, hipStream_t st);
// Event timing of one launch sequence of a profiled part (no-op unless enabled).
int timed_part(Plan& p, int part, double flops, hipStream_t st, const std::function<int()>& launch);
int check_batch(const Plan& p, long batch);
int fill_f64(double* x, long n, double v, hipStream_t st);
int fill_i32(int32_t* x, long n, int32_t v, hipStream_t st);
int fill_i64(int64_t* x, long n, int64_t v, hipStream_t st);
int copy_f64(const double* a, double* b, long n, hipStream_t st);
int copy_i8(const int8_t* a, int8_t* b, long n, hipStream_t st);

// Local sweeps
int launch_flip_slice(Plan& p, int batch, int8_t* s, double* G, double* logabs, int8_t* sign, int slice,
                      uint64_t seed, uint64_t sweep, uint64_t chain0, int64_t* accepts, hipStream_t st);
int launch_drift(Plan& p, int batch, double* Gw, const double* Gf, double* drift, int32_t* status, hipStream_t st);
int sweep_stacked(Plan& p, int batch, int8_t* s, double* G, double* logabs, int8_t* sign, int n_sweeps,
                  uint64_t seed, uint64_t sweep0, uint64_t chain0, int64_t* accepts, double* drift,
                  int32_t* status, hipStream_t st);
size_t stack_bytes_for(const Plan& p, long batch);  // bytes of the stacked partial products

// Effective model
int launch_eff_sweep(Plan& p, const Eff& e, int batch, int8_t* s, int n_moves, uint64_t seed, uint64_t step,
                     uint64_t chain0, int64_t* accepts, double* dS, hipStream_t st);
int launch_features(Plan& p, const Eff& e, long count, const int8_t* s, double* F, hipStream_t st);
int launch_accept(Plan& p, const Eff& e, int batch, int8_t* s, const int8_t* sprop, double* logabs, int8_t* sign,
                  const double* new_logabs, const int8_t* new_sign, const double* F_old, const double* F_new,
                  const double* Sn_old, const double* Sn_new, uint64_t seed, uint64_t step, uint64_t chain0,
                  int8_t* accepted, double* logA, hipStream_t st);
int launch_fit_chunked(Plan& p, const Eff& e, long n, const int8_t* s, const double* y, double* theta, double* r2,
                       hipStream_t st);

// Learned action
int net_forward(Plan& p, int prec, int batch, const int8_t* s, const double* prm, double* S, hipStream_t st);
int launch_eff_sweep_net(Plan& p, const Eff& e, int batch, int8_t* s, int n_moves, uint64_t seed, uint64_t step,
                         uint64_t chain0, int64_t* accepts, double* dS, hipStream_t st);
int net_pair(Plan& p, const Eff& e, int batch, const int8_t* s_old, const int8_t* s_new, double** old_out,
             double** new_out, hipStream_t st);
void release_net(Plan& p);               // frees the host view only
size_t net_bytes_for(const Plan& p);     // device bytes of the network buffers for max_batch fields
int bind_net(Plan& p);                   // host view of the buffers at p.net_base

// Workspace layout and set-up shared by plan creation and the size query.
constexpr long FIT_ACC_DOUBLES = 2 * (MAX_TERMS_ABI + 2) * (MAX_TERMS_ABI + 2);
size_t plan_layout(Plan& p, int32_t flags, char* base);
int plan_init(Plan& p, hipStream_t st);

}  // namespace slq

struct slq_plan {
  slq::Plan p;
};
struct slq_eff {
  slq::Eff e;
};
