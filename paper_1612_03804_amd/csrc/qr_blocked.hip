// Blocked Householder QR of a batch of pre-pivoted matrices, MFMA trailing
// updates (the stabilisation step of the slice-matrix chain; see qr.hip for
// the factorisation that is computed and why).
//
// For each panel of NB columns:
//   k_panel   one workgroup per field factors the m x NB panel in LDS
//             (LAPACK dlarfg convention, H = I - tau v v^T, beta = -sign(alpha)
//             ||x||), forms the compact-WY factor T (Q_p = I - V T V^T), and
//             writes V explicitly and T;
//   GEMM      Wt  = V^T A_trail                     (K = m, MFMA)
//   GEMM      Wt2 = T^T Wt                          (K = NB)
//   GEMM      A_trail -= V Wt2                      (K = NB, MFMA)
// and the explicit Q = Q_1 ... Q_P is accumulated backwards with the same
// three GEMMs (T in place of T^T).  The column pre-pivoting (sort by norm of
// X diag(D_prev)) and the permuted, scaled copy run in k_prepivot.
#include <algorithm>

#include "slq_internal.h"

namespace slq {

constexpr int PQ_THREADS = 512;
constexpr int PQ_WAVES = PQ_THREADS / 64;

__device__ __forceinline__ double pq_block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < PQ_WAVES; ++w) t += red[w];
  return t;
}

__device__ __forceinline__ double pq_block_max(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < PQ_WAVES; ++w) t = fmax(t, red[w]);
  return t;
}

// ------------------------------------------------------------ prepivot ----
// perm = columns of X diag(D) by decreasing norm (lower index first on
// ties); W[:, c] = X[:, perm[c]] * D[perm[c]].
__global__ __launch_bounds__(PQ_THREADS) void k_prepivot(int N, const double* __restrict__ Xall,
                                                         double* __restrict__ Wall, const double* __restrict__ Dall,
                                                         int32_t* __restrict__ permall, int32_t* status) {
  extern __shared__ double lds[];
  const int b = blockIdx.x;
  const long NN = (long)N * N;
  const double* X = Xall + b * NN;
  double* W = Wall + b * NN;
  const double* D = Dall + (long)b * N;
  int32_t* perm = permall + (long)b * N;
  double* nrm = lds;
  int* rp = (int*)(lds + N);
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int j = threadIdx.x; j < N; j += PQ_THREADS) {
    double ss = 0.0, mx = 0.0;
    for (int i = 0; i < N; ++i) {
      const double v = X[(long)i * N + j];
      ss += v * v;
      mx = fmax(mx, fabs(v));
    }
    double nv = sqrt(ss);
    if (!(nv < INFINITY) || (nv < 1e-150 && mx > 0.0)) {  // rescale when the plain sum over/underflows
      ss = 0.0;
      const double inv = 1.0 / mx;
      for (int i = 0; i < N; ++i) {
        const double v = X[(long)i * N + j] * inv;
        ss += v * v;
      }
      nv = mx * sqrt(ss);
    }
    nv *= fabs(D[j]);
    if (!(nv >= 0.0) || isinf(nv)) {
      nv = -1.0;
      bad = 1;
    }
    nrm[j] = nv;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < N; j += PQ_THREADS) {
    const double nj = nrm[j];
    int r = 0;
    for (int i = 0; i < N; ++i) {
      const double ni = nrm[i];
      r += (ni > nj) || (ni == nj && i < j);
    }
    rp[r] = j;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < N; c += PQ_THREADS) perm[c] = rp[c];
  for (long idx = threadIdx.x; idx < NN; idx += PQ_THREADS) {
    const int i = (int)(idx / N), c = (int)(idx % N);
    const int pc = rp[c];
    W[idx] = X[(long)i * N + pc] * D[pc];
  }
  if (threadIdx.x == 0 && bad && status) atomicOr(&status[b], SLQ_ST_NONFINITE);
}

// --------------------------------------------------------------- panel ----
struct PanelArgs {
  int N, j0, nbw;
  double* W;       // [b][N][N]: panel columns j0..j0+nbw, rows j0..N-1 (in: A, out: R above / V below)
  double* Vbuf;    // [b][N][N]: explicit V of the panel at rows j0.., columns j0..j0+NB
  double* T;       // [b] + strideT: compact-WY factor of this panel, [NB][NB] row-major
  long strideT;
  double* D;       // [b][N] out: |R_jj|
  double* invD;    // [b][N] out: 1/|R_jj|
  int32_t* nref;   // [b] in/out: reflectors with tau != 0
  int32_t* status;
};

// One workgroup per field factors the m x nbw panel.  Wave w owns the
// columns c = w (mod waves) and keeps them in registers, row r = lane + 64 k
// in slot k (RPL slots cover m).  Step c: the owner of column c has formed
// reflector c (LAPACK dlarfg: beta = -sign(alpha) ||x||, v = x / (alpha -
// beta) below the diagonal) and published v_c in LDS; after one barrier every
// wave applies H_c = I - tau_c v_c v_c^T to its own columns > c (the owner of
// column c+1 first, and it forms reflector c+1 at once) and adds the Gram
// entries v_i . v_c of its finished columns i < c.  T (Q_panel = I - V T V^T)
// follows from the Gram matrix at the end.
template <int NB, int RPL, bool CACHE_V>
__global__ __launch_bounds__(PQ_THREADS) void k_panel(PanelArgs a) {
  extern __shared__ double lds[];
  constexpr int CPW = NB >= PQ_WAVES ? NB / PQ_WAVES : 1;  // columns per wave
  constexpr int LT = NB + 1;        // padded row stride of T and the Gram matrix
  const int N = a.N, j0 = a.j0, nbw = a.nbw, m = N - j0;
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long NN = (long)N * N;
  double* W = a.W + b * NN;
  const int ldp = m + 1;            // column stride of the panel in LDS
  double* P = lds;                  // [NB][ldp]: staging, then the published reflectors
  double* T = P + (long)NB * ldp;   // [NB][LT]
  double* Gm = T + NB * LT;         // [NB][LT]
  double* tau = Gm + NB * LT;       // [NB]

  for (int r = tid / NB; r < m; r += PQ_THREADS / NB) {
    const int c = tid % NB;
    if (c < nbw) P[c * ldp + r] = W[(long)(j0 + r) * N + j0 + c];
  }
  __syncthreads();
  double col[CPW][RPL];
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int c = wave + PQ_WAVES * q;
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
      const int r = lane + 64 * k;
      col[q][k] = (c < nbw && r < m) ? P[c * ldp + r] : 0.0;
    }
  }
  __syncthreads();  // the staging area is reused for the reflectors

  // reflector of the owned column q, global column c (uniform)
  auto reflect = [&](int q, int c) {
    double ss = 0.0, mx = 0.0, alpha = 0.0;
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
      const int r = lane + 64 * k;
      const double v = col[q][k];
      if (r > c && r < m) {
        ss += v * v;
        mx = fmax(mx, fabs(v));
      }
      if (k == c / 64) alpha = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), c % 64),
                                                __builtin_amdgcn_readlane(__double2loint(v), c % 64));
    }
    double xnorm = sqrt(wave_sum(ss));
    if (!(xnorm < INFINITY) || xnorm < 1e-150) {  // rescale when the plain sum over/underflows
      mx = wave_max(mx);
      if (mx > 0.0) {
        const double inv = 1.0 / mx;
        double s2 = 0.0;
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
          const int r = lane + 64 * k;
          const double v = col[q][k] * inv;
          if (r > c && r < m) s2 += v * v;
        }
        xnorm = mx * sqrt(wave_sum(s2));
      } else {
        xnorm = 0.0;
      }
    }
    double tc = 0.0, beta = alpha;
    if (xnorm > 0.0) {
      beta = -copysign(hypot(alpha, xnorm), alpha);
      tc = (beta - alpha) / beta;
      const double scal = 1.0 / (alpha - beta);
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        const int r = lane + 64 * k;
        if (r > c && r < m) col[q][k] *= scal;
      }
    }
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
      const int r = lane + 64 * k;
      if (r == c) col[q][k] = beta;
      if (r > c && r < m) P[c * ldp + r] = col[q][k];
    }
    if (lane == 0) tau[c] = tc;
  };

  if (wave == 0) reflect(0, 0);
  for (int c = 0; c < nbw; ++c) {
    __syncthreads();  // reflector c is published; step c - 1 is done everywhere
    const double tc = tau[c];
    double vr[CACHE_V ? RPL : 1];
    auto vrow = [&](int k) -> double {  // v_c at row lane + 64 k
      const int r = lane + 64 * k;
      return r < c || r >= m ? 0.0 : (r == c ? 1.0 : P[c * ldp + r]);
    };
    if (CACHE_V) {
#pragma unroll
      for (int k = 0; k < RPL; ++k) vr[k] = vrow(k);
    }
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      const int c2 = wave + PQ_WAVES * q;
      if (c2 >= nbw) continue;
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < RPL; ++k) s += (CACHE_V ? vr[k] : vrow(k)) * col[q][k];
      s = wave_sum(s);
      if (c2 > c) {  // apply H_c
        if (tc != 0.0) {
          s *= tc;
#pragma unroll
          for (int k = 0; k < RPL; ++k) col[q][k] -= s * (CACHE_V ? vr[k] : vrow(k));
        }
        if (c2 == c + 1) reflect(q, c2);
      } else if (c2 < c) {  // finished column: Gram entry v_{c2} . v_c
        if (lane == 0) Gm[c2 * LT + c] = s;
      }
    }
  }
  __syncthreads();  // the last reflector has been read everywhere
  // owned columns back to LDS: R above the diagonal, V below
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int c = wave + PQ_WAVES * q;
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
      const int r = lane + 64 * k;
      if (c < nbw && r < m) P[c * ldp + r] = col[q][k];
    }
  }
  __syncthreads();
  if (wave == 0) {
    // T[0:j, j] = -tau_j T[0:j, 0:j] Gm[0:j, j], T[j][j] = tau_j, in registers:
    // lane i holds row i of T and row i of the Gram matrix; Gm[k][j] reaches
    // every lane as a lane read of lane k
    const bool live = lane < nbw;
    double trow[NB], grow[NB];
    const double tl = live ? tau[lane] : 0.0;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      grow[j] = (live && lane < j && j < nbw) ? Gm[lane * LT + j] : 0.0;
      trow[j] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (j < nbw) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < j; ++k) s += trow[k] * read_lane(grow[j], k);
        const double tj = read_lane(tl, j);
        trow[j] = lane < j ? -tj * s : (lane == j ? tj : 0.0);
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j)
      if (lane < NB) T[lane * LT + j] = live && j < nbw ? trow[j] : 0.0;
    const double d = live ? fabs(P[lane * ldp + lane]) : 1.0;
    const unsigned long long refl = __ballot(live && tau[lane] != 0.0);
    const unsigned long long bad = __ballot(live && (!(d > 0.0) || !(d < INFINITY)));
    if (live) {
      a.D[(long)b * N + j0 + lane] = d;
      a.invD[(long)b * N + j0 + lane] = 1.0 / d;
    }
    if (lane == 0) {
      a.nref[b] += __popcll(refl);
      if (bad && a.status) atomicOr(&a.status[b], SLQ_ST_NONFINITE);
    }
  }
  __syncthreads();
  // R and V back into W; explicit V (unit diagonal, zeros above); T
  double* Vb = a.Vbuf + b * NN;
  for (int r = tid / NB; r < m; r += PQ_THREADS / NB) {
    const int c = tid % NB;
    if (c < nbw) {
      const double pv = P[c * ldp + r];
      W[(long)(j0 + r) * N + j0 + c] = pv;
      Vb[(long)(j0 + r) * N + j0 + c] = (r == c) ? 1.0 : (r > c ? pv : 0.0);
    }
  }
  double* Tg = a.T + b * a.strideT;
  for (int idx = tid; idx < NB * NB; idx += PQ_THREADS) Tg[idx] = T[(idx / NB) * LT + idx % NB];
}

// panel width and register rows per lane by matrix size
template <int NB>
struct PanelShape;
template <>
struct PanelShape<32> {
  static constexpr int RPL = 7;  // N <= 448
  static constexpr bool CACHE = true;
};
template <>
struct PanelShape<16> {
  static constexpr int RPL = 18;  // N <= 1152
  static constexpr bool CACHE = true;
};
template <>
struct PanelShape<8> {
  static constexpr int RPL = 38;  // N <= 2432
  static constexpr bool CACHE = false;
};

__global__ void k_zero_i32(int32_t* x, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x[i] = 0;
}

template <int NB>
static int run_blocked(Plan& p, int batch, const double* X, const UdvRef& o, int32_t* status, hipStream_t st) {
  const int N = p.n;
  const long NN = (long)N * N;
  const int npanel = (N + NB - 1) / NB;
  // scratch: Vbuf = Xb-or-Xa not holding X (both are free once W is written),
  // T per panel, Wt = V^T A and Wt2 = T^T Wt (or T Wt)
  double* Vbuf = (X == p.Xa) ? p.Xb : p.Xa;
  double* Tb = p.Tblk;  // [b][npanel][NB][NB]
  const long strideT = (long)npanel * NB * NB;
  double* Wt = p.dY;    // [b][NB][N]
  double* Wt2 = p.dX;   // [b][NB][N]
  const size_t lpp = sizeof(double) * N + sizeof(int) * N;
  allow_max_lds((const void*)k_prepivot);
  k_prepivot<<<batch, PQ_THREADS, lpp, st>>>(N, X, p.W, o.D, p.perm, status);
  SLQ_LAUNCHED();
  k_zero_i32<<<(batch + 255) / 256, 256, 0, st>>>(o.nref, batch);
  SLQ_LAUNCHED();
  // Wt = V^T B;  Wt2 = op(T) Wt;  B -= V Wt2   (B: m x n block at row/col j0, col jc)
  auto apply = [&](int j0, int nbw, int m, double* Bblk, int n, bool transT, double* Tp) -> int {
    GemmArgs g1{};
    g1.M = nbw;
    g1.N = n;
    g1.K = m;
    g1.A = Vbuf + (long)j0 * N + j0;
    g1.lda = N;
    g1.strideA = NN;
    g1.B = Bblk;
    g1.ldb = N;
    g1.strideB = NN;
    g1.C = Wt;
    g1.ldc = N;
    g1.strideC = (long)NB * N;
    g1.alpha = 1.0;
    g1.batch = batch;
    int rc = launch_gemm(g1, true, false, st);
    if (rc != SLQ_OK) return rc;
    GemmArgs gt{};
    gt.M = nbw;
    gt.N = n;
    gt.K = nbw;
    gt.A = Tp;
    gt.lda = NB;
    gt.strideA = strideT;
    gt.B = Wt;
    gt.ldb = N;
    gt.strideB = (long)NB * N;
    gt.C = Wt2;
    gt.ldc = N;
    gt.strideC = (long)NB * N;
    gt.alpha = 1.0;
    gt.batch = batch;
    rc = launch_gemm(gt, transT, false, st);
    if (rc != SLQ_OK) return rc;
    GemmArgs g2{};
    g2.M = m;
    g2.N = n;
    g2.K = nbw;
    g2.A = Vbuf + (long)j0 * N + j0;
    g2.lda = N;
    g2.strideA = NN;
    g2.B = Wt2;
    g2.ldb = N;
    g2.strideB = (long)NB * N;
    g2.C = Bblk;
    g2.ldc = N;
    g2.strideC = NN;
    g2.alpha = -1.0;
    g2.beta = 1.0;
    g2.batch = batch;
    return launch_gemm(g2, false, false, st);
  };
  for (int pi = 0; pi < npanel; ++pi) {
    const int j0 = pi * NB, nbw = std::min(NB, N - j0), m = N - j0, nt = N - j0 - nbw;
    PanelArgs a{N, j0, nbw, p.W, Vbuf, Tb + (long)pi * NB * NB, strideT, o.D, p.invD, o.nref, status};
    const size_t lds = sizeof(double) * ((size_t)NB * (m + 1) + 2 * NB * (NB + 1) + NB);
    constexpr int RPL = PanelShape<NB>::RPL;
    constexpr bool CACHE = PanelShape<NB>::CACHE;
    allow_max_lds((const void*)k_panel<NB, RPL, CACHE>);
    k_panel<NB, RPL, CACHE><<<batch, PQ_THREADS, lds, st>>>(a);
    SLQ_LAUNCHED();
    if (nt <= 0) continue;
    // A_trail <- Q_p^T A_trail = A_trail - V (T^T (V^T A_trail))
    int rc = apply(j0, nbw, m, p.W + (long)j0 * N + j0 + nbw, nt, true, Tb + (long)pi * NB * NB);
    if (rc != SLQ_OK) return rc;
  }
  // explicit Q, backwards: U[j0:, j0:] <- Q_p U[j0:, j0:] = U - V (T (V^T U))
  int rc = launch_set_identity(p, batch, o.U, st);
  if (rc != SLQ_OK) return rc;
  for (int pi = npanel - 1; pi >= 0; --pi) {
    const int j0 = pi * NB, nbw = std::min(NB, N - j0), m = N - j0;
    rc = apply(j0, nbw, m, o.U + (long)j0 * N + j0, m, false, Tb + (long)pi * NB * NB);
    if (rc != SLQ_OK) return rc;
  }
  return SLQ_OK;
}

int qr_blocked_width(int N) { return N <= 448 ? 32 : (N <= 1152 ? 16 : 8); }

int launch_qr_blocked(Plan& p, int batch, const double* X, const UdvRef& o, int32_t* status, hipStream_t st) {
  switch (qr_blocked_width(p.n)) {
    case 32: return run_blocked<32>(p, batch, X, o, status, st);
    case 16: return run_blocked<16>(p, batch, X, o, status, st);
    default: return run_blocked<8>(p, batch, X, o, status, st);
  }
}

}  // namespace slq
