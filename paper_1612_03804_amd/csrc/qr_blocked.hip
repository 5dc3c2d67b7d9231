// Blocked Householder QR of a batch of pre-pivoted matrices, MFMA trailing
// updates (the stabilisation step of the slice-matrix chain; see qr.hip for
// the factorisation that is computed and why).
//
// For each panel of NB columns:
//   k_panel   one workgroup per field factors the m x NB panel in LDS
//             (LAPACK dlarfg convention, H = I - tau v v^T, beta = -sign(alpha)
//             ||x||), forms the compact-WY factor T (Q_p = I - V T V^T), and
//             writes V explicitly together with Y = V T^T and Z = V T;
//   GEMM      Wt = V^T A_trail                      (K = m, MFMA)
//   GEMM      A_trail -= Y Wt                       (K = NB, MFMA)
// and the explicit Q = Q_1 ... Q_P is accumulated backwards with the same two
// GEMMs (Z in place of Y).  The column pre-pivoting (sort by norm of
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
  double* Zbuf;    // [b][N][N]: Z = V T at the same place
  double* Ybuf;    // [b][N][NB]: Y = V T^T, rows 0..m-1
  double* D;       // [b][N] out: |R_jj|
  double* invD;    // [b][N] out: 1/|R_jj|
  int32_t* nref;   // [b] in/out: reflectors with tau != 0
  int32_t* status;
};

template <int NB>
__global__ __launch_bounds__(PQ_THREADS) void k_panel(PanelArgs a) {
  extern __shared__ double lds[];
  const int N = a.N, j0 = a.j0, nbw = a.nbw, m = N - j0;
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long NN = (long)N * N;
  double* W = a.W + b * NN;
  const int ldp = m + 1;         // column stride of the panel in LDS
  double* P = lds;               // [NB][ldp]
  double* T = P + (long)NB * ldp;  // [NB][NB]
  double* Gm = T + NB * NB;        // [NB][NB] Gram of the reflectors
  double* tau = Gm + NB * NB;      // [NB]
  double* wv = tau + NB;           // [NB]
  double* red = wv + NB;           // [PQ_WAVES]

  for (int idx = tid; idx < m * nbw; idx += PQ_THREADS) {
    const int c = idx % nbw, r = idx / nbw;
    P[c * ldp + r] = W[(long)(j0 + r) * N + j0 + c];
  }
  __syncthreads();
  int nref = 0;
  bool bad = false;
  for (int c = 0; c < nbw; ++c) {
    double ss = 0.0, mx = 0.0;
    for (int r = c + 1 + tid; r < m; r += PQ_THREADS) {
      const double v = P[c * ldp + r];
      ss += v * v;
      mx = fmax(mx, fabs(v));
    }
    ss = pq_block_sum(ss, red);
    double xnorm = sqrt(ss);
    if (!(xnorm < INFINITY) || xnorm < 1e-150) {
      mx = pq_block_max(mx, red);
      if (mx > 0.0) {
        const double inv = 1.0 / mx;
        double s2 = 0.0;
        for (int r = c + 1 + tid; r < m; r += PQ_THREADS) {
          const double v = P[c * ldp + r] * inv;
          s2 += v * v;
        }
        s2 = pq_block_sum(s2, red);
        xnorm = mx * sqrt(s2);
      } else {
        xnorm = 0.0;
      }
    }
    const double alpha = P[c * ldp + c];
    double tc = 0.0, beta = alpha;
    if (xnorm > 0.0) {
      beta = -copysign(hypot(alpha, xnorm), alpha);
      tc = (beta - alpha) / beta;
      const double scal = 1.0 / (alpha - beta);
      for (int r = c + 1 + tid; r < m; r += PQ_THREADS) P[c * ldp + r] *= scal;
    }
    if (!(fabs(beta) > 0.0) || !(fabs(beta) < INFINITY)) bad = true;
    nref += (tc != 0.0);
    __syncthreads();
    if (tid == 0) {
      P[c * ldp + c] = beta;
      tau[c] = tc;
    }
    if (tc != 0.0 && c + 1 < nbw) {
      for (int c2 = c + 1 + wave; c2 < nbw; c2 += PQ_WAVES) {
        double s = 0.0;
        for (int r = c + 1 + lane; r < m; r += 64) s += P[c * ldp + r] * P[c2 * ldp + r];
        s = wave_sum(s);
        if (lane == 0) wv[c2] = tc * (s + P[c2 * ldp + c]);
      }
      __syncthreads();
      const int w2 = nbw - c - 1;
      for (int idx = tid; idx < w2 * (m - c); idx += PQ_THREADS) {
        const int c2 = c + 1 + idx % w2;
        const int r = c + idx / w2;
        const double v = (r == c) ? 1.0 : P[c * ldp + r];
        P[c2 * ldp + r] -= wv[c2] * v;
      }
    }
    __syncthreads();
  }
  // Gram of the reflectors (unit diagonal, zero above) and T
  for (int pr = wave; pr < nbw * nbw; pr += PQ_WAVES) {
    const int i = pr / nbw, j = pr % nbw;
    if (i < j) {
      double s = 0.0;
      for (int r = j + 1 + lane; r < m; r += 64) s += P[i * ldp + r] * P[j * ldp + r];
      s = wave_sum(s);
      if (lane == 0) Gm[i * NB + j] = s + P[i * ldp + j];
    }
  }
  for (int idx = tid; idx < NB * NB; idx += PQ_THREADS) T[idx] = 0.0;
  __syncthreads();
  for (int j = 0; j < nbw; ++j) {
    if (tid < j) {
      double s = 0.0;
      for (int k = tid; k < j; ++k) s += T[tid * NB + k] * Gm[k * NB + j];
      T[tid * NB + j] = -tau[j] * s;
    }
    if (tid == j) T[j * NB + j] = tau[j];
    __syncthreads();
  }
  // outputs: R and V back into W; explicit V, Y = V T^T, Z = V T
  double* Vb = a.Vbuf + b * NN;
  double* Zb = a.Zbuf + b * NN;
  double* Yb = a.Ybuf + (long)b * N * NB;
  for (int idx = tid; idx < m * nbw; idx += PQ_THREADS) {
    const int c = idx % nbw, r = idx / nbw;
    W[(long)(j0 + r) * N + j0 + c] = P[c * ldp + r];
    const double v = (r == c) ? 1.0 : (r > c ? P[c * ldp + r] : 0.0);
    // Y[r][c] = sum_k V[r][k] T[c][k];  Z[r][c] = sum_k V[r][k] T[k][c]
    double y = 0.0, z = 0.0;
    const int kmax = min(r, nbw - 1);
    for (int k = 0; k <= kmax; ++k) {
      const double vk = (r == k) ? 1.0 : P[k * ldp + r];
      y += vk * T[c * NB + k];
      z += vk * T[k * NB + c];
    }
    Vb[(long)(j0 + r) * N + j0 + c] = v;
    Zb[(long)(j0 + r) * N + j0 + c] = z;
    Yb[(long)r * NB + c] = y;
  }
  for (int c = tid; c < nbw; c += PQ_THREADS) {
    const double d = fabs(P[c * ldp + c]);
    a.D[(long)b * N + j0 + c] = d;
    a.invD[(long)b * N + j0 + c] = 1.0 / d;
  }
  if (tid == 0) {
    a.nref[b] += nref;
    if (bad && a.status) atomicOr(&a.status[b], SLQ_ST_NONFINITE);
  }
}

__global__ void k_zero_i32(int32_t* x, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x[i] = 0;
}

template <int NB>
static int run_blocked(Plan& p, int batch, const double* X, const UdvRef& o, int32_t* status, hipStream_t st) {
  const int N = p.n;
  const long NN = (long)N * N;
  // scratch: Vbuf = Xb-or-Xa not holding X (both are free once W is written), Y, Wt
  double* Vbuf = (X == p.Xa) ? p.Xb : p.Xa;
  double* Zbuf = p.Vt;  // Vt is rebuilt after the QR from V and perm
  double* Ybuf = p.dX;  // [b][N][NB] (local-sweep scratch is idle here)
  double* Wt = p.dY;    // [b][NB][N]
  const size_t lpp = sizeof(double) * N + sizeof(int) * N;
  allow_max_lds((const void*)k_prepivot);
  k_prepivot<<<batch, PQ_THREADS, lpp, st>>>(N, X, p.W, o.D, p.perm, status);
  SLQ_LAUNCHED();
  k_zero_i32<<<(batch + 255) / 256, 256, 0, st>>>(o.nref, batch);
  SLQ_LAUNCHED();
  const int npanel = (N + NB - 1) / NB;
  for (int pi = 0; pi < npanel; ++pi) {
    const int j0 = pi * NB, nbw = std::min(NB, N - j0), m = N - j0, nt = N - j0 - nbw;
    PanelArgs a{N, j0, nbw, p.W, Vbuf, Zbuf, Ybuf, o.D, p.invD, o.nref, status};
    const size_t lds = sizeof(double) * ((size_t)NB * (m + 1) + 2 * NB * NB + 2 * NB + PQ_WAVES);
    allow_max_lds((const void*)k_panel<NB>);
    k_panel<NB><<<batch, PQ_THREADS, lds, st>>>(a);
    SLQ_LAUNCHED();
    if (nt <= 0) continue;
    GemmArgs g1{};  // Wt = V^T A_trail
    g1.M = nbw;
    g1.N = nt;
    g1.K = m;
    g1.A = Vbuf + (long)j0 * N + j0;
    g1.lda = N;
    g1.strideA = NN;
    g1.B = p.W + (long)j0 * N + j0 + nbw;
    g1.ldb = N;
    g1.strideB = NN;
    g1.C = Wt;
    g1.ldc = N;
    g1.strideC = (long)NB * N;
    g1.alpha = 1.0;
    g1.batch = batch;
    int rc = launch_gemm(g1, true, false, st);
    if (rc != SLQ_OK) return rc;
    GemmArgs g2{};  // A_trail -= Y Wt
    g2.M = m;
    g2.N = nt;
    g2.K = nbw;
    g2.A = Ybuf;
    g2.lda = NB;
    g2.strideA = (long)N * NB;
    g2.B = Wt;
    g2.ldb = N;
    g2.strideB = (long)NB * N;
    g2.C = p.W + (long)j0 * N + j0 + nbw;
    g2.ldc = N;
    g2.strideC = NN;
    g2.alpha = -1.0;
    g2.beta = 1.0;
    g2.batch = batch;
    rc = launch_gemm(g2, false, false, st);
    if (rc != SLQ_OK) return rc;
  }
  // explicit Q, backwards: U[j0:, j0:] -= Z (V^T U[j0:, j0:])
  int rc = launch_set_identity(p, batch, o.U, st);
  if (rc != SLQ_OK) return rc;
  for (int pi = npanel - 1; pi >= 0; --pi) {
    const int j0 = pi * NB, nbw = std::min(NB, N - j0), m = N - j0;
    GemmArgs g1{};
    g1.M = nbw;
    g1.N = m;
    g1.K = m;
    g1.A = Vbuf + (long)j0 * N + j0;
    g1.lda = N;
    g1.strideA = NN;
    g1.B = o.U + (long)j0 * N + j0;
    g1.ldb = N;
    g1.strideB = NN;
    g1.C = Wt;
    g1.ldc = N;
    g1.strideC = (long)NB * N;
    g1.alpha = 1.0;
    g1.batch = batch;
    rc = launch_gemm(g1, true, false, st);
    if (rc != SLQ_OK) return rc;
    GemmArgs g2{};
    g2.M = m;
    g2.N = m;
    g2.K = nbw;
    g2.A = Zbuf + (long)j0 * N + j0;
    g2.lda = N;
    g2.strideA = NN;
    g2.B = Wt;
    g2.ldb = N;
    g2.strideB = (long)NB * N;
    g2.C = o.U + (long)j0 * N + j0;
    g2.ldc = N;
    g2.strideC = NN;
    g2.alpha = -1.0;
    g2.beta = 1.0;
    g2.batch = batch;
    rc = launch_gemm(g2, false, false, st);
    if (rc != SLQ_OK) return rc;
  }
  return SLQ_OK;
}

int qr_blocked_width(int N) { return N <= 448 ? 32 : (N <= 1100 ? 16 : 8); }

int launch_qr_blocked(Plan& p, int batch, const double* X, const UdvRef& o, int32_t* status, hipStream_t st) {
  switch (qr_blocked_width(p.n)) {
    case 32: return run_blocked<32>(p, batch, X, o, status, st);
    case 16: return run_blocked<16>(p, batch, X, o, status, st);
    default: return run_blocked<8>(p, batch, X, o, status, st);
  }
}

}  // namespace slq
