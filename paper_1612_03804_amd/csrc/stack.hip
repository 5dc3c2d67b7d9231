// Local DQMC sweeps with stabilised partial products kept between the
// periodic recomputations of G (section "Basics of DQMC": one flip costs
// O(1) for the ratio and O(N^2) for the update, a sweep O(beta N^3)).
//
// At a boundary b (a multiple of n_stab) the sweep needs
//     G_b = (1 + R(b) Left(b))^{-1},   R(b) = B_b ... B_1,   Left(b) = B_L ... B_{b+1}.
// Both factors are kept as stabilised products U D V:
//   R(b)        is extended block by block as the sweep moves up, from slices
//               whose fields the sweep has already visited;
//   Left(b)^T = B_{b+1}^T ... B_L^T  is built for every boundary at the start
//               of the sweep (B_l^T = diag(d_l) E because E is symmetric), from
//               slices the sweep has not reached yet.
// With Left(b) = V_L^T D_L U_L^T and the pre-pivoted QR
//     diag(D_R) (V_R V_L^T) diag(D_L) = Q D (D^{-1} R) Pi^T
// one gets 1 + R(b) Left(b) = 1 + (U_R Q) D ((D^{-1} R) Pi^T U_L^T), a product
// of the same shape the final step of a weight evaluation turns into G, its
// log-determinant and its sign (det U_R Q is the parity of both reflection
// counts).  A sweep then costs about 2L slice products and 3L/n_stab QRs
// instead of the L^2/n_stab products of recomputing the whole cyclic chain
// at every boundary.
#include <algorithm>

#include "slq_internal.h"

namespace slq {

// X = B_l^T = diag(d_l) E (rows of E scaled by the field of slice l).
__global__ void k_first_slice_rows(int N, const double* __restrict__ E, const int8_t* __restrict__ s, long strideS,
                                   int slice, const double* __restrict__ consts, double* __restrict__ X) {
  const int b = blockIdx.y;
  const long NN = (long)N * N;
  const int8_t* sb = s + (long)b * strideS + (long)slice * N;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < NN; idx += (long)gridDim.x * blockDim.x) {
    const int i = (int)(idx / N);
    X[b * NN + idx] = E[idx] * (sb[i] > 0 ? consts[0] : consts[1]);
  }
}

// Vt = Pi^T U^T: Vt[c][j] = U[j][perm[c]].
__global__ void k_permute_cols_t(int N, const double* __restrict__ U, const int32_t* __restrict__ perm,
                                 double* __restrict__ Vt) {
  const long NN = (long)N * N;
  const int b = blockIdx.y;
  const int32_t* pb = perm + (long)b * N;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < NN; idx += (long)gridDim.x * blockDim.x) {
    const int c = (int)(idx / N), j = (int)(idx % N);
    Vt[b * NN + idx] = U[b * NN + (long)j * N + pb[c]];
  }
}

__global__ void k_add_i32(int32_t* a, const int32_t* __restrict__ b, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] += b[i];
}

static dim3 grid_nn(const Plan& p, int batch) {
  const long NN = (long)p.n * p.n;
  return dim3((unsigned)std::min<long>((NN + 255) / 256, 1024), batch);
}

// Number of boundaries strictly below L: the entries of the left stack.
static int n_left(const Plan& p) { return (p.L - 1) / p.m.n_stab; }

size_t stack_bytes_for(const Plan& p, long batch) {
  const long N = p.n;
  return sizeof(double) * (size_t)(n_left(p) + 1) * batch * (2 * N * N + N) + sizeof(int32_t) * batch;
}

// Entry e < n_left: Left((e+1) n_stab)^T.  Entry n_left: the running R(b),
// the only one whose reflection count is kept (the left ones write theirs to
// the plan's scratch: det U_L does not enter G_b).
static UdvRef entry(Plan& p, int e) {
  const long N = p.n, NN = N * N, B = p.stack_batch;
  const int nl = n_left(p);
  double* base = p.stack + (size_t)e * B * (2 * NN + N);
  int32_t* nref = e == nl ? (int32_t*)(p.stack + (size_t)(nl + 1) * B * (2 * NN + N)) : p.nref;
  return UdvRef{base, base + 2 * B * NN, base + B * NN, nref};
}

static int need_stack(const Plan& p) {
  if (p.stack) return SLQ_OK;
  set_error("the plan was created without SLQ_PLAN_SWEEPS (no room for the stacked partial products)");
  return SLQ_ERR_WORKSPACE;
}

// Product of the count slices first, first + step, ... (0-based), the first
// one applied first, onto `start` (the identity when start is null).  Plain:
// X <- B_l X = E diag(d_l) X.  Transposed: X <- B_l^T X = diag(d_l) E X.
// Returns the buffer (Xa or Xb) that holds the result, and in *norm2 the
// squared column norms of it when the structured product computed them
// (else null).
static int block_product(Plan& p, int batch, const int8_t* s, int first, int count, int step, bool transposed,
                         const double* start, double** out, const double** norm2, hipStream_t st) {
  *norm2 = nullptr;
  const int N = p.n;
  const long NN = (long)N * N;
  const long strideS = (long)p.L * N;
  if (has_structured(p)) {  // structured products, the whole block in one launch
    KronArgs k{};
    k.in = start;
    k.strideIn = NN;
    k.out = p.Xa;
    k.strideOut = NN;
    k.s = s;
    k.slice0 = first;
    k.count = count;
    k.step = step;
    k.scale = transposed ? 2 : 1;
    k.batch = batch;
    k.norm2 = p.xnorm2;
    *out = p.Xa;
    *norm2 = p.xnorm2;
    return launch_kron(p, k, st);
  }
  GemmArgs g{};
  g.M = N;
  g.N = N;
  g.K = N;
  g.A = p.E;
  g.lda = N;
  g.ldb = N;
  g.strideB = NN;
  g.ldc = N;
  g.strideC = NN;
  g.S = s;
  g.strideS = strideS;
  g.consts = p.consts;
  g.alpha = 1.0;
  g.s_out = transposed ? 1 : 0;
  g.cfg = p.gemm_cfg;
  g.batch = batch;
  double* cur = p.Xa;
  double* oth = p.Xb;
  int k = 0;
  if (!start) {
    if (transposed) {
      k_first_slice_rows<<<grid_nn(p, batch), 256, 0, st>>>(N, p.E, s, strideS, first, p.consts, cur);
      SLQ_LAUNCHED();
    } else {
      SLQ_TRY(launch_first_slice(p, batch, s, strideS, first, cur, st));
    }
    k = 1;
  } else {
    g.B = start;
    g.C = cur;
    g.slice = first;
    SLQ_TRY(launch_gemm(g, false, false, st));
    k = 1;
  }
  for (; k < count; ++k) {
    g.B = cur;
    g.C = oth;
    g.slice = first + k * step;
    SLQ_TRY(launch_gemm(g, false, false, st));
    std::swap(cur, oth);
  }
  *out = cur;
  return SLQ_OK;
}

// X diag(D_in) = Q D (D^{-1} R) Pi^T, then out = (Q, D, (D^{-1} R) Pi^T V_in).
// D_in and V_in null mean the identity; D_in may be out.D and V_in out.V.
// X (Xa or Xb) is destroyed.
static int stabilise(Plan& p, int batch, double* X, const double* D_in, const double* V_in, const UdvRef& out,
                     int32_t* status, hipStream_t st, const double* norm2 = nullptr) {
  const int N = p.n;
  const long NN = (long)N * N;
  if (!D_in)
    SLQ_TRY(fill_f64(out.D, (long)batch * N, 1.0, st));
  else if (D_in != out.D)
    SLQ_TRY(copy_f64(D_in, out.D, (long)batch * N, st));
  if (N > 64)
    SLQ_TRY(launch_qr_blocked(p, batch, X, out, status, st, norm2));
  else
    SLQ_TRY(launch_qr(p, batch, X, out, status, st));
  if (!V_in) return launch_first_v(p, batch, out.V, st);
  if (V_in != out.V) return launch_v_update(p, batch, V_in, out.V, st);
  SLQ_TRY(copy_f64(V_in, p.Vt, (long)batch * NN, st));  // in place: read from a copy
  return launch_v_update(p, batch, p.Vt, out.V, st);
}

// Left(b)^T for every boundary b < L, from the top of the chain down.
static int build_left(Plan& p, int batch, const int8_t* s, int32_t* status, hipStream_t st) {
  const int L = p.L, ns = p.m.n_stab, nl = n_left(p);
  for (int e = nl - 1; e >= 0; --e) {
    const int b = (e + 1) * ns;                     // slices b+1 .. top, applied top first
    const int top = (e == nl - 1) ? L : b + ns;     // 1-based
    const UdvRef out = entry(p, e);
    double* X = nullptr;
    const double* n2 = nullptr;
    if (e == nl - 1) {
      SLQ_TRY(block_product(p, batch, s, top - 1, top - b, -1, true, nullptr, &X, &n2, st));
      SLQ_TRY(stabilise(p, batch, X, nullptr, nullptr, out, status, st, n2));
    } else {
      const UdvRef prev = entry(p, e + 1);
      SLQ_TRY(block_product(p, batch, s, top - 1, top - b, -1, true, prev.U, &X, &n2, st));
      SLQ_TRY(stabilise(p, batch, X, prev.D, prev.V, out, status, st, n2));
    }
  }
  return SLQ_OK;
}

// R(b) = B_b ... B_{b-ns+1} R(b - ns), in place in the right entry.
static int extend_right(Plan& p, int batch, const int8_t* s, int b, int32_t* status, hipStream_t st) {
  const int ns = p.m.n_stab;
  const UdvRef r = entry(p, n_left(p));
  double* X = nullptr;
  const double* n2 = nullptr;
  if (b == ns) {
    SLQ_TRY(block_product(p, batch, s, 0, ns, 1, false, nullptr, &X, &n2, st));
    return stabilise(p, batch, X, nullptr, nullptr, r, status, st, n2);
  }
  SLQ_TRY(block_product(p, batch, s, b - ns, ns, 1, false, r.U, &X, &n2, st));
  return stabilise(p, batch, X, r.D, r.V, r, status, st, n2);
}

// Fresh G_b into p.Xa from R(b) and Left(b) (b < L), or from R(L) alone.
static int fresh_green(Plan& p, int batch, int b, int32_t* status, hipStream_t st) {
  const int N = p.n, nl = n_left(p);
  const long NN = (long)N * N;
  const UdvRef r = entry(p, nl);
  if (b == p.L) return launch_finish(p, batch, r, p.Xa, p.dvec, p.sgn_work, status, st);
  const UdvRef lf = entry(p, b / p.m.n_stab - 1);
  GemmArgs x{};  // Xa = diag(D_R) V_R V_L^T
  x.M = N;
  x.N = N;
  x.K = N;
  x.A = r.V;
  x.lda = N;
  x.strideA = NN;
  x.B = lf.V;
  x.ldb = N;
  x.strideB = NN;
  x.C = p.Xa;
  x.ldc = N;
  x.strideC = NN;
  x.rowscale = r.D;
  x.strideRS = N;
  x.alpha = 1.0;
  x.batch = batch;
  SLQ_TRY(launch_gemm(x, false, true, st));
  const UdvRef m{p.U, p.D, p.V, p.nref};
  SLQ_TRY(copy_f64(lf.D, m.D, (long)batch * N, st));
  if (N > 64)
    SLQ_TRY(launch_qr_blocked(p, batch, p.Xa, m, status, st));
  else
    SLQ_TRY(launch_qr(p, batch, p.Xa, m, status, st));
  GemmArgs u{};  // Xb = U_R Q
  u.M = N;
  u.N = N;
  u.K = N;
  u.A = r.U;
  u.lda = N;
  u.strideA = NN;
  u.B = m.U;
  u.ldb = N;
  u.strideB = NN;
  u.C = p.Xb;
  u.ldc = N;
  u.strideC = NN;
  u.alpha = 1.0;
  u.batch = batch;
  SLQ_TRY(launch_gemm(u, false, false, st));
  k_permute_cols_t<<<grid_nn(p, batch), 256, 0, st>>>(N, lf.U, p.perm, p.Vt);
  SLQ_LAUNCHED();
  GemmArgs v{};  // V = (D^{-1} R) Pi^T U_L^T
  v.M = N;
  v.N = N;
  v.K = N;
  v.A = p.W;
  v.lda = N;
  v.strideA = NN;
  v.B = p.Vt;
  v.ldb = N;
  v.strideB = NN;
  v.C = m.V;
  v.ldc = N;
  v.strideC = NN;
  v.rowscale = p.invD;
  v.strideRS = N;
  v.alpha = 1.0;
  v.a_upper = 1;
  v.batch = batch;
  SLQ_TRY(launch_gemm(v, false, false, st));
  k_add_i32<<<(batch + 255) / 256, 256, 0, st>>>(m.nref, r.nref, batch);
  SLQ_LAUNCHED();
  return launch_finish(p, batch, UdvRef{p.Xb, m.D, m.V, m.nref}, p.Xa, p.dvec, p.sgn_work, status, st);
}

int sweep_stacked(Plan& p, int batch, int8_t* s, double* G, double* logabs, int8_t* sign, int n_sweeps,
                  uint64_t seed, uint64_t sweep0, uint64_t chain0, int64_t* accepts, double* drift,
                  int32_t* status, hipStream_t st) {
  const int N = p.n, L = p.L, ns = p.m.n_stab;
  const long NN = (long)N * N;
  SLQ_TRY(need_stack(p));
  GemmArgs w1{};  // Xa = E diag(d_l) G
  w1.M = N;
  w1.N = N;
  w1.K = N;
  w1.A = p.E;
  w1.lda = N;
  w1.B = G;
  w1.ldb = N;
  w1.strideB = NN;
  w1.C = p.Xa;
  w1.ldc = N;
  w1.strideC = NN;
  w1.S = s;
  w1.strideS = (long)L * N;
  w1.consts = p.consts;
  w1.alpha = 1.0;
  w1.batch = batch;
  GemmArgs w2 = w1;  // G = Xa diag(1/d_l) E^{-1}
  w2.A = p.Xa;
  w2.strideA = NN;
  w2.B = p.Einv;
  w2.strideB = 0;
  w2.C = G;
  w2.inv_scale = 1;
  KronArgs k1{};  // Xa = E diag(d_l) G, on the columns
  k1.in = G;
  k1.strideIn = NN;
  k1.out = p.Xa;
  k1.strideOut = NN;
  k1.s = s;
  k1.count = 1;
  k1.step = 1;
  k1.scale = 1;
  k1.batch = batch;
  KronArgs k2 = k1;  // G = Xa diag(1/d_l) E^{-1}: each row r -> E^{-1} diag(1/d_l) r
  k2.in = p.Xa;
  k2.out = G;
  k2.rows = 1;
  k2.inv = 1;
  for (int k = 0; k < n_sweeps; ++k) {
    if (L > ns) SLQ_TRY(build_left(p, batch, s, status, st));
    for (int l = 1; l <= L; ++l) {
      SLQ_TRY(launch_flip_slice(p, batch, s, G, logabs, sign, l - 1, seed, sweep0 + k, chain0, accepts, st));
      if (has_structured(p)) {
        k1.slice0 = l - 1;
        k2.slice0 = l - 1;
        SLQ_TRY(launch_kron(p, k1, st));
        SLQ_TRY(launch_kron(p, k2, st));
      } else {
        w1.slice = l - 1;
        w2.slice = l - 1;
        SLQ_TRY(launch_gemm(w1, false, false, st));
        SLQ_TRY(launch_gemm(w2, false, false, st));
      }
      if (l % ns == 0) {
        SLQ_TRY(extend_right(p, batch, s, l, status, st));
        SLQ_TRY(fresh_green(p, batch, l, status, st));
        SLQ_TRY(launch_drift(p, batch, G, p.Xa, drift, status, st));
      }
    }
  }
  return SLQ_OK;
}

}  // namespace slq
