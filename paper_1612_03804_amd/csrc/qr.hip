// Stabilisation of the slice-matrix chain: column-pre-pivoted blocked
// Householder QR of X diag(D_prev), one workgroup per field.
//
// The paper relies on the standard numerically stabilised DQMC algorithm
// (cited in its Introduction for the O(beta N^3) cost) without describing
// it.  The partial product is kept as U diag(D) V; after n_stab new slices
// X = B...B U and
//     X diag(D) Pi = Q R,   U <- Q,   D <- |diag R|,   V <- diag(1/D) R Pi^T V.
// Pi sorts the columns of X diag(D) by decreasing Euclidean norm
// ("pre-pivoting"); the graded scales D then appear in decreasing order on the
// diagonal of R as with LAPACK's column-pivoted QR, while the factorisation
// itself is the blocked Householder QR with compact-WY panels
// (Q_p = I - V_p T_p V_p^T).  The determinant and G do not depend on the
// choice of pivots.
//
// Work per call: norms, ranks and the permuted copy (O(N^2)), panel
// factorisation in LDS, trailing updates streamed through L2 with one
// column per thread and NB accumulators in registers, and the explicit Q by
// backward accumulation of the panels.
#include "slq_internal.h"

namespace slq {

constexpr int QR_THREADS = 512;
constexpr int QR_WAVES = QR_THREADS / 64;

struct QrArgs {
  int N;
  const double* X;  // [batch][N][N] chain product
  double* W;        // [batch][N][N] out: R (upper) and Householder vectors (lower)
  double* U;        // [batch][N][N] out: Q
  double* D;        // [batch][N] in: D_prev, out: D_new = |diag R|
  double* invD;     // [batch][N] out: 1 / D_new
  int32_t* perm;    // [batch][N] out: column order
  double* Tblk;     // [batch][npanel][NB][NB] compact-WY T factors
  int32_t* nref;    // [batch] out: number of reflectors with tau != 0
  int32_t* status;  // [batch] |= SLQ_ST_NONFINITE
};

__device__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < QR_WAVES; ++w) t += red[w];
  return t;
}

__device__ double block_max(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < QR_WAVES; ++w) t = fmax(t, red[w]);
  return t;
}

// Householder vectors of panel (j0, nbw) live in LDS as P[c*ldp + r],
// r = 0..m-1 relative to row j0, with the unit diagonal and zero upper part
// implicit.  apply_panel() computes, for columns [jbeg, N) of the row-major
// matrix Mx (rows j0..N-1), Mx <- (I - V op(T) V^T) Mx, op(T) = T^T when
// transT (Q^T applied from the left) and T otherwise (Q from the left).
template <int NB>
__device__ void apply_panel(double* __restrict__ Mx, int N, int j0, int nbw, int jbeg, const double* P, int ldp,
                            const double* T, bool transT) {
  const int m = N - j0;
  for (int j = jbeg + threadIdx.x; j < N; j += QR_THREADS) {
    double w[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) w[c] = 0.0;
    // rows in the unit-triangle part: r < nbw
    for (int r = 0; r < nbw; ++r) {
      const double a = Mx[(long)(j0 + r) * N + j];
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c < nbw) {
          const double v = (r == c) ? 1.0 : (r > c ? P[c * ldp + r] : 0.0);
          w[c] += v * a;
        }
      }
    }
    for (int r = nbw; r < m; ++r) {
      const double a = Mx[(long)(j0 + r) * N + j];
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nbw) w[c] += P[c * ldp + r] * a;
    }
    double y[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      double s = 0.0;
      if (c < nbw) {
        if (transT) {
          for (int k = 0; k <= c; ++k) s += T[k * NB + c] * w[k];
        } else {
          for (int k = c; k < nbw; ++k) s += T[c * NB + k] * w[k];
        }
      }
      y[c] = s;
    }
    for (int r = 0; r < nbw; ++r) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c < nbw) {
          const double v = (r == c) ? 1.0 : (r > c ? P[c * ldp + r] : 0.0);
          s += v * y[c];
        }
      }
      Mx[(long)(j0 + r) * N + j] -= s;
    }
    for (int r = nbw; r < m; ++r) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nbw) s += P[c * ldp + r] * y[c];
      Mx[(long)(j0 + r) * N + j] -= s;
    }
  }
}

template <int NB>
__global__ __launch_bounds__(QR_THREADS) void k_qr(QrArgs a) {
  extern __shared__ double lds[];
  const int N = a.N;
  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long NN = (long)N * N;
  const double* X = a.X + b * NN;
  double* W = a.W + b * NN;
  double* U = a.U + b * NN;
  double* D = a.D + (long)b * N;
  double* invD = a.invD + (long)b * N;
  int32_t* perm = a.perm + (long)b * N;
  const int npanel = (N + NB - 1) / NB;
  double* Tg = a.Tblk + (long)b * npanel * NB * NB;

  const int ldp = N;
  double* P = lds;                       // [NB][N] panel
  double* T = lds + (long)NB * N;        // [NB][NB]
  double* Y = T + NB * NB;               // [NB][NB] Gram of the panel vectors
  double* tau = Y + NB * NB;             // [NB]
  double* red = tau + NB;                // [QR_WAVES]
  double* wv = red + QR_WAVES;           // [NB]
  int* flag = (int*)(wv + NB);           // [2]

  if (tid == 0) {
    flag[0] = 0;
    flag[1] = 0;
  }
  __syncthreads();

  // ---- 1. norms of the columns of X diag(D_prev)
  double* nrm = P;
  int* rank_perm = (int*)(P + N);
  for (int j = tid; j < N; j += QR_THREADS) {
    double mx = 0.0;
    for (int i = 0; i < N; ++i) mx = fmax(mx, fabs(X[(long)i * N + j]));
    double s = 0.0;
    if (mx > 0.0) {
      const double inv = 1.0 / mx;
      for (int i = 0; i < N; ++i) {
        const double v = X[(long)i * N + j] * inv;
        s += v * v;
      }
    }
    double nv = fabs(D[j]) * mx * sqrt(s);
    if (!(nv >= 0.0) || isinf(nv)) {
      nv = -1.0;
      atomicOr(&flag[0], 1);
    }
    nrm[j] = nv;
  }
  __syncthreads();
  // ---- 2. ranks: decreasing norm, lower index first on ties
  for (int j = tid; j < N; j += QR_THREADS) {
    const double nj = nrm[j];
    int r = 0;
    for (int i = 0; i < N; ++i) {
      const double ni = nrm[i];
      r += (ni > nj) || (ni == nj && i < j);
    }
    rank_perm[r] = j;
  }
  __syncthreads();
  for (int c = tid; c < N; c += QR_THREADS) perm[c] = rank_perm[c];
  // ---- 3. W[:, c] = X[:, perm[c]] * D_prev[perm[c]]
  for (long idx = tid; idx < NN; idx += QR_THREADS) {
    const int i = (int)(idx / N), c = (int)(idx % N);
    const int pc = rank_perm[c];
    W[idx] = X[(long)i * N + pc] * D[pc];
  }
  __syncthreads();

  // ---- 4. blocked Householder QR of W in place
  int nref = 0;
  for (int p = 0; p < npanel; ++p) {
    const int j0 = p * NB;
    const int nbw = min(NB, N - j0);
    const int m = N - j0;
    for (int idx = tid; idx < m * nbw; idx += QR_THREADS) {
      const int c = idx % nbw, r = idx / nbw;
      P[c * ldp + r] = W[(long)(j0 + r) * N + j0 + c];
    }
    __syncthreads();
    for (int c = 0; c < nbw; ++c) {
      // tail norm of column c below the diagonal, scaled against overflow
      double mx = 0.0;
      for (int r = c + 1 + tid; r < m; r += QR_THREADS) mx = fmax(mx, fabs(P[c * ldp + r]));
      mx = block_max(mx, red);
      double ss = 0.0;
      if (mx > 0.0) {
        const double inv = 1.0 / mx;
        for (int r = c + 1 + tid; r < m; r += QR_THREADS) {
          const double v = P[c * ldp + r] * inv;
          ss += v * v;
        }
      }
      ss = block_sum(ss, red);
      const double xnorm = mx * sqrt(ss);
      const double alpha = P[c * ldp + c];
      double tc = 0.0, beta = alpha;
      if (xnorm > 0.0) {
        beta = -copysign(hypot(alpha, xnorm), alpha);
        tc = (beta - alpha) / beta;
        const double scal = 1.0 / (alpha - beta);
        for (int r = c + 1 + tid; r < m; r += QR_THREADS) P[c * ldp + r] *= scal;
      }
      __syncthreads();
      if (tid == 0) {
        P[c * ldp + c] = beta;
        tau[c] = tc;
      }
      if (tc != 0.0) ++nref;
      // apply H_c to the remaining panel columns
      if (tc != 0.0) {
        for (int c2 = c + 1 + wave; c2 < nbw; c2 += QR_WAVES) {
          double s = 0.0;
          for (int r = c + 1 + lane; r < m; r += 64) s += P[c * ldp + r] * P[c2 * ldp + r];
          s = wave_sum(s);
          if (lane == 0) wv[c2] = s + P[c2 * ldp + c];
        }
        __syncthreads();
        for (int idx = tid; idx < (nbw - c - 1) * (m - c); idx += QR_THREADS) {
          const int c2 = c + 1 + idx % (nbw - c - 1);
          const int r = c + idx / (nbw - c - 1);
          const double v = (r == c) ? 1.0 : P[c * ldp + r];
          P[c2 * ldp + r] -= tc * wv[c2] * v;
        }
      }
      __syncthreads();
    }
    // Gram Y[i][j] = v_i . v_j (i < j) and the compact-WY factor T
    for (int pr = wave; pr < nbw * nbw; pr += QR_WAVES) {
      const int i = pr / nbw, j = pr % nbw;
      if (i < j) {
        double s = 0.0;
        for (int r = j + 1 + lane; r < m; r += 64) s += P[i * ldp + r] * P[j * ldp + r];
        s = wave_sum(s);
        if (lane == 0) Y[i * NB + j] = s + P[i * ldp + j];
      }
    }
    for (int idx = tid; idx < NB * NB; idx += QR_THREADS) T[idx] = 0.0;
    __syncthreads();
    for (int j = 0; j < nbw; ++j) {
      // T[0:j, j] = -tau_j T[0:j, 0:j] Y[0:j, j];  T[j][j] = tau_j
      if (tid < j) {
        double s = 0.0;
        for (int k = tid; k < j; ++k) s += T[tid * NB + k] * Y[k * NB + j];
        T[tid * NB + j] = -tau[j] * s;
      }
      if (tid == j) T[j * NB + j] = tau[j];
      __syncthreads();
    }
    for (int idx = tid; idx < NB * NB; idx += QR_THREADS) Tg[(long)p * NB * NB + idx] = T[idx];
    // write the factored panel back
    for (int idx = tid; idx < m * nbw; idx += QR_THREADS) {
      const int c = idx % nbw, r = idx / nbw;
      W[(long)(j0 + r) * N + j0 + c] = P[c * ldp + r];
    }
    // trailing update W[j0:, j0+nbw:] <- Q_p^T W[j0:, j0+nbw:]
    apply_panel<NB>(W, N, j0, nbw, j0 + nbw, P, ldp, T, true);
    __syncthreads();
  }

  // ---- D = |diag R|
  for (int i = tid; i < N; i += QR_THREADS) {
    const double d = fabs(W[(long)i * N + i]);
    if (!(d > 0.0) || isinf(d)) atomicOr(&flag[0], 1);
    D[i] = d;
    invD[i] = 1.0 / d;
  }

  // ---- 5. explicit Q by backward accumulation of the panels
  for (long idx = tid; idx < NN; idx += QR_THREADS) U[idx] = ((idx / N) == (idx % N)) ? 1.0 : 0.0;
  __syncthreads();
  for (int p = npanel - 1; p >= 0; --p) {
    const int j0 = p * NB;
    const int nbw = min(NB, N - j0);
    const int m = N - j0;
    for (int idx = tid; idx < m * nbw; idx += QR_THREADS) {
      const int c = idx % nbw, r = idx / nbw;
      P[c * ldp + r] = W[(long)(j0 + r) * N + j0 + c];
    }
    for (int idx = tid; idx < NB * NB; idx += QR_THREADS) T[idx] = Tg[(long)p * NB * NB + idx];
    __syncthreads();
    apply_panel<NB>(U, N, j0, nbw, j0, P, ldp, T, false);
    __syncthreads();
  }
  if (tid == 0) {
    a.nref[b] = nref;
    if (flag[0] && a.status) a.status[b] |= SLQ_ST_NONFINITE;
  }
}

static size_t qr_lds(int N, int nb) {
  return sizeof(double) * ((size_t)nb * N + 2 * nb * nb + nb + QR_WAVES + nb) + 2 * sizeof(int);
}

int qr_panel_width(int N) { return N <= 1024 ? 16 : 8; }

int launch_qr(Plan& p, int batch, const double* X, const UdvRef& o, int32_t* status, hipStream_t st) {
  QrArgs a;
  a.N = p.n;
  a.X = X;
  a.W = p.W;
  a.U = o.U;
  a.D = o.D;
  a.invD = p.invD;
  a.perm = p.perm;
  a.Tblk = p.Tblk;
  a.nref = o.nref;
  a.status = status;
  const int nb = qr_panel_width(p.n);
  const size_t lds = qr_lds(p.n, nb);
  if (nb == 16) {
    allow_max_lds((const void*)k_qr<16>);
    k_qr<16><<<batch, QR_THREADS, lds, st>>>(a);
  } else {
    allow_max_lds((const void*)k_qr<8>);
    k_qr<8><<<batch, QR_THREADS, lds, st>>>(a);
  }
  SLQ_LAUNCHED();
  return SLQ_OK;
}

// ------------------------------------------------------------- helpers ----
__global__ void k_first_slice(int N, const double* __restrict__ E, const int8_t* __restrict__ s, long strideS,
                              int slice, const double* __restrict__ consts, double* __restrict__ X) {
  const int b = blockIdx.y;
  const long NN = (long)N * N;
  const int8_t* sb = s + (long)b * strideS + (long)slice * N;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < NN; idx += (long)gridDim.x * blockDim.x) {
    const int j = (int)(idx % N);
    X[b * NN + idx] = E[idx] * (sb[j] > 0 ? consts[0] : consts[1]);
  }
}

int launch_first_slice(Plan& p, int batch, const int8_t* s, long strideS, int slice, double* X, hipStream_t st) {
  const long NN = (long)p.n * p.n;
  dim3 grid((unsigned)std::min<long>((NN + 255) / 256, 1024), batch);
  k_first_slice<<<grid, 256, 0, st>>>(p.n, p.E, s, strideS, slice, p.consts, X);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

__global__ void k_set_identity(int N, double* X) {
  const long NN = (long)N * N;
  const int b = blockIdx.y;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < NN; idx += (long)gridDim.x * blockDim.x)
    X[b * NN + idx] = (idx / N == idx % N) ? 1.0 : 0.0;
}

int launch_set_identity(Plan& p, int batch, double* X, hipStream_t st) {
  const long NN = (long)p.n * p.n;
  dim3 grid((unsigned)std::min<long>((NN + 255) / 256, 1024), batch);
  k_set_identity<<<grid, 256, 0, st>>>(p.n, X);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

// V_prev = I: V[i][j] = R[i][c] / D_i where perm[c] = j, zero for c < i
// (diag(1/D) triu(R) Pi^T).  One workgroup per 8 rows of a field; the inverse
// permutation in LDS makes the writes coalesced.
constexpr int FV_ROWS = 8;
__global__ __launch_bounds__(256) void k_first_v(int N, const double* __restrict__ W, const double* __restrict__ invD,
                                                 const int32_t* __restrict__ perm, double* __restrict__ V) {
  extern __shared__ int cinv[];  // [N]
  const int b = blockIdx.y, r0 = blockIdx.x * FV_ROWS;
  const long NN = (long)N * N;
  for (int c = threadIdx.x; c < N; c += blockDim.x) cinv[perm[(long)b * N + c]] = c;
  __syncthreads();
  const int rows = min(FV_ROWS, N - r0);
  for (int e = threadIdx.x; e < rows * N; e += blockDim.x) {
    const int i = r0 + e / N, j = e % N;
    const int c = cinv[j];
    V[b * NN + (long)i * N + j] = c >= i ? W[b * NN + (long)i * N + c] * invD[(long)b * N + i] : 0.0;
  }
}

int launch_first_v(Plan& p, int batch, double* V, hipStream_t st) {
  dim3 grid((unsigned)((p.n + FV_ROWS - 1) / FV_ROWS), (unsigned)batch);
  k_first_v<<<grid, 256, sizeof(int) * p.n, st>>>(p.n, p.W, p.invD, p.perm, V);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

int launch_v_update(Plan& p, int batch, const double* V_in, double* V_out, hipStream_t st) {
  const int N = p.n;
  const long NN = (long)N * N;
  GemmArgs v{};  // V_out <- diag(1/D) triu(R) (Pi^T V_in), Pi^T applied while B is read
  v.M = N;
  v.N = N;
  v.K = N;
  v.A = p.W;
  v.lda = N;
  v.strideA = NN;
  v.B = V_in;
  v.ldb = N;
  v.strideB = NN;
  v.brow = p.perm;
  v.strideBrow = N;
  v.C = V_out;
  v.ldc = N;
  v.strideC = NN;
  v.rowscale = p.invD;
  v.strideRS = N;
  v.alpha = 1.0;
  v.beta = 0.0;
  v.a_upper = 1;
  v.batch = batch;
  // large tile-aligned N: 128 x 128 tiles of 64 x 64 per wavefront (N = 2304,
  // 256 fields: 60.6 against 62.2 ms per update on 64 x 128 tiles); otherwise
  // columns up to the last multiple of 128 on 64 x 128 tiles, a 16-column
  // remainder on 128 x 16 tiles (no padded columns)
  const int Nm = N / 128 * 128;
  if (N > 1152 && Nm == N) {
    v.cfg = GEMM_BIG;
    return launch_gemm(v, false, false, st);
  }
  if (Nm == 0 || Nm == N || (N - Nm) % 16 != 0) return launch_gemm(v, false, false, st);
  v.N = Nm;
  v.cfg = GEMM_64x128;
  SLQ_TRY(launch_gemm(v, false, false, st));
  v.N = N - Nm;
  v.B = V_in + Nm;
  v.C = V_out + Nm;
  v.cfg = (N - Nm) <= 16 ? GEMM_128x16 : GEMM_64x128;
  return launch_gemm(v, false, false, st);
}

__global__ void k_check_spins(long total_per_item, const int8_t* __restrict__ s, int32_t* status) {
  const int b = blockIdx.y;
  const int8_t* sb = s + (long)b * total_per_item;
  int bad = 0;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total_per_item;
       idx += (long)gridDim.x * blockDim.x) {
    const int v = sb[idx];
    bad |= (v != 1 && v != -1);
  }
  if (bad) atomicOr(&status[b], SLQ_ST_BAD_SPIN);
}

int launch_check_spins(Plan& p, int batch, const int8_t* s, int32_t* status, hipStream_t st) {
  const long per = (long)p.n * p.L;
  dim3 grid((unsigned)std::min<long>((per + 255) / 256, 64), batch);
  k_check_spins<<<grid, 256, 0, st>>>(per, s, status);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

}  // namespace slq
