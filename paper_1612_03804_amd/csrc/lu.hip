// Final step of the stabilised evaluation: log|det(1 + U D V)|, its sign and
// G = (1 + U D V)^{-1}, one workgroup per field.
//
// With D_b = max(D, 1) and D_s = min(D, 1),
//     1 + U D V = U D_b M,   M = D_b^{-1} U^T + D_s V,
// so det(1 + B_L...B_1) = det(U) prod(D_b) det(M) (the determinant of Eq. 1;
// the paper counts this step as the O(N^3) cost of calculating the
// determinant) and G = M^{-1} D_b^{-1} U^T.  M is well conditioned: the large
// scales sit in D_b^{-1} <= 1 and the small ones in D_s <= 1.  det U = +-1
// from the number of Householder reflectors; det M from an LU factorisation
// with partial pivoting (blocked, panel in LDS, right-looking updates with
// one column per thread).
#include "slq_internal.h"

namespace slq {

constexpr int FN_THREADS = 512;
constexpr int FN_WAVES = FN_THREADS / 64;

struct FinishArgs {
  int N;
  const double* U;
  const double* D;
  const double* V;
  const int32_t* nref;
  double* W;
  int32_t* ipiv;
  double* G;  // may be null
  double* logabs;
  int8_t* sign;
  int32_t* status;
};

// out[i][j] = scale_i * src[j][i]  (+ add_i * addm[i][j] when addm != null), tiled through LDS.
__device__ void transpose_scaled(int N, const double* __restrict__ src, const double* __restrict__ D,
                                 const double* __restrict__ addm, double* __restrict__ out, double* tile) {
  constexpr int TS = 32;
  const int nt = (N + TS - 1) / TS;
  for (int t = 0; t < nt * nt; ++t) {
    const int ti = t / nt, tj = t % nt;  // output tile rows i in ti, columns j in tj
    __syncthreads();
    for (int e = threadIdx.x; e < TS * TS; e += FN_THREADS) {
      const int r = e / TS, c = e % TS;  // src row j = tj*TS + r, col i = ti*TS + c
      const int j = tj * TS + r, i = ti * TS + c;
      tile[r * (TS + 1) + c] = (j < N && i < N) ? src[(long)j * N + i] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < TS * TS; e += FN_THREADS) {
      const int r = e / TS, c = e % TS;  // out row i = ti*TS + r, col j = tj*TS + c
      const int i = ti * TS + r, j = tj * TS + c;
      if (i < N && j < N) {
        const double d = D[i];
        double v = tile[c * (TS + 1) + r] / fmax(d, 1.0);
        if (addm) v += fmin(d, 1.0) * addm[(long)i * N + j];
        out[(long)i * N + j] = v;
      }
    }
  }
  __syncthreads();
}

template <int NB>
__global__ __launch_bounds__(FN_THREADS) void k_finish(FinishArgs a) {
  extern __shared__ double lds[];
  const int N = a.N;
  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long NN = (long)N * N;
  const double* U = a.U + b * NN;
  const double* V = a.V + b * NN;
  const double* D = a.D + (long)b * N;
  double* W = a.W + b * NN;
  int32_t* ipiv = a.ipiv + (long)b * N;

  double* P = lds;                    // [NB][N] panel, or the 32 x 33 transpose tile
  double* redv = P + max(NB * N, 32 * 33);  // [FN_WAVES]
  int* redi = (int*)(redv + FN_WAVES);  // [FN_WAVES]
  int* flag = redi + FN_WAVES;          // [2]
  if (tid == 0) flag[0] = 0;
  __syncthreads();

  // ---- M = D_b^{-1} U^T + D_s V
  transpose_scaled(N, U, D, V, W, P);

  // ---- LU with partial pivoting, in place
  const int ldp = N;
  for (int j0 = 0; j0 < N; j0 += NB) {
    const int nbw = min(NB, N - j0);
    const int m = N - j0;
    for (int idx = tid; idx < m * nbw; idx += FN_THREADS) {
      const int c = idx % nbw, r = idx / nbw;
      P[c * ldp + r] = W[(long)(j0 + r) * N + j0 + c];
    }
    __syncthreads();
    for (int c = 0; c < nbw; ++c) {
      double best = -1.0;
      int bi = m;
      for (int r = c + tid; r < m; r += FN_THREADS) {
        const double v = fabs(P[c * ldp + r]);
        if (v > best) {
          best = v;
          bi = r;
        }
      }
      wave_argmax(best, bi);
      if (lane == 0) {
        redv[wave] = best;
        redi[wave] = bi;
      }
      __syncthreads();
      best = redv[0];
      bi = redi[0];
      for (int w = 1; w < FN_WAVES; ++w)
        if (redv[w] > best || (redv[w] == best && redi[w] < bi)) {
          best = redv[w];
          bi = redi[w];
        }
      const bool zero = !(best > 0.0);
      const int piv = zero ? c : bi;
      if (tid == 0) {
        ipiv[j0 + c] = j0 + piv;
        if (zero) flag[0] = 1;
      }
      if (piv != c && tid < nbw) {
        const double t = P[tid * ldp + c];
        P[tid * ldp + c] = P[tid * ldp + piv];
        P[tid * ldp + piv] = t;
      }
      __syncthreads();
      if (!zero) {
        const double inv = 1.0 / P[c * ldp + c];
        for (int r = c + 1 + tid; r < m; r += FN_THREADS) P[c * ldp + r] *= inv;
        __syncthreads();
        const int w2 = nbw - c - 1;
        if (w2 > 0)
          for (int idx = tid; idx < w2 * (m - c - 1); idx += FN_THREADS) {
            const int c2 = c + 1 + idx % w2;
            const int r = c + 1 + idx / w2;
            P[c2 * ldp + r] -= P[c * ldp + r] * P[c2 * ldp + c];
          }
      }
      __syncthreads();
    }
    for (int idx = tid; idx < m * nbw; idx += FN_THREADS) {
      const int c = idx % nbw, r = idx / nbw;
      W[(long)(j0 + r) * N + j0 + c] = P[c * ldp + r];
    }
    // columns outside the panel: row swaps, then U12 = L11^{-1} A12 and the
    // trailing update A22 -= L21 U12 (one column per thread)
    for (int j = tid; j < N; j += FN_THREADS) {
      if (j >= j0 && j < j0 + nbw) continue;
      for (int c = 0; c < nbw; ++c) {
        const int pr = ipiv[j0 + c];
        if (pr != j0 + c) {
          const double t = W[(long)(j0 + c) * N + j];
          W[(long)(j0 + c) * N + j] = W[(long)pr * N + j];
          W[(long)pr * N + j] = t;
        }
      }
      if (j < j0 + nbw) continue;
      double x[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) x[c] = (c < nbw) ? W[(long)(j0 + c) * N + j] : 0.0;
#pragma unroll
      for (int c = 1; c < NB; ++c)
        if (c < nbw)
          for (int c2 = 0; c2 < c; ++c2) x[c] -= P[c2 * ldp + c] * x[c2];
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nbw) W[(long)(j0 + c) * N + j] = x[c];
      for (int r = nbw; r < m; ++r) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c < nbw) s += P[c * ldp + r] * x[c];
        W[(long)(j0 + r) * N + j] -= s;
      }
    }
    __syncthreads();
  }

  // ---- log|det| and sign (fixed reduction order: deterministic)
  double lsum = 0.0;
  int par = 0;
  for (int i = tid; i < N; i += FN_THREADS) {
    const double u = W[(long)i * N + i];
    lsum += log(fabs(u)) + log(fmax(D[i], 1.0));
    par ^= (u < 0.0) ^ (ipiv[i] != i);
  }
  lsum = wave_sum(lsum);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) par ^= __shfl_xor(par, o, 64);
  __syncthreads();
  if (lane == 0) {
    redv[wave] = lsum;
    redi[wave] = par;
  }
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    int pp = a.nref[b] & 1;
    for (int w = 0; w < FN_WAVES; ++w) {
      tot += redv[w];
      pp ^= redi[w];
    }
    const bool sing = flag[0] != 0;
    if (sing && a.status) a.status[b] |= SLQ_ST_SINGULAR;
    if (!isfinite(tot) && !sing && a.status) a.status[b] |= SLQ_ST_NONFINITE;
    a.logabs[b] = sing ? -INFINITY : tot;
    a.sign[b] = sing ? 0 : (pp ? -1 : 1);
  }
  if (!a.G) return;

  // ---- G = M^{-1} D_b^{-1} U^T
  double* G = a.G + b * NN;
  transpose_scaled(N, U, D, nullptr, G, P);
  // row swaps (each thread owns whole columns, so no barrier is needed)
  for (int j = tid; j < N; j += FN_THREADS)
    for (int k = 0; k < N; ++k) {
      const int pr = ipiv[k];
      if (pr != k) {
        const double t = G[(long)k * N + j];
        G[(long)k * N + j] = G[(long)pr * N + j];
        G[(long)pr * N + j] = t;
      }
    }
  __syncthreads();
  // forward substitution with the unit lower factor
  for (int i0 = 0; i0 < N; i0 += NB) {
    const int nbw = min(NB, N - i0);
    const int m = N - i0;
    for (int idx = tid; idx < m * nbw; idx += FN_THREADS) {
      const int c = idx % nbw, r = idx / nbw;
      P[c * ldp + r] = W[(long)(i0 + r) * N + i0 + c];
    }
    __syncthreads();
    for (int j = tid; j < N; j += FN_THREADS) {
      double x[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) x[c] = (c < nbw) ? G[(long)(i0 + c) * N + j] : 0.0;
#pragma unroll
      for (int c = 1; c < NB; ++c)
        if (c < nbw)
          for (int c2 = 0; c2 < c; ++c2) x[c] -= P[c2 * ldp + c] * x[c2];
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nbw) G[(long)(i0 + c) * N + j] = x[c];
      for (int r = nbw; r < m; ++r) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c < nbw) s += P[c * ldp + r] * x[c];
        G[(long)(i0 + r) * N + j] -= s;
      }
    }
    __syncthreads();
  }
  // backward substitution with the upper factor
  const int nblk = (N + NB - 1) / NB;
  for (int blk = nblk - 1; blk >= 0; --blk) {
    const int i0 = blk * NB;
    const int nbw = min(NB, N - i0);
    const int rows = i0 + nbw;  // U rows 0 .. i0+nbw-1 of columns i0 .. i0+nbw-1
    for (int idx = tid; idx < rows * nbw; idx += FN_THREADS) {
      const int c = idx % nbw, r = idx / nbw;
      P[c * ldp + r] = W[(long)r * N + i0 + c];
    }
    __syncthreads();
    for (int j = tid; j < N; j += FN_THREADS) {
      double x[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) x[c] = (c < nbw) ? G[(long)(i0 + c) * N + j] : 0.0;
#pragma unroll
      for (int c = NB - 1; c >= 0; --c)
        if (c < nbw) {
          double s = x[c];
          for (int c2 = c + 1; c2 < nbw; ++c2) s -= P[c2 * ldp + i0 + c] * x[c2];
          x[c] = s / P[c * ldp + i0 + c];
        }
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nbw) G[(long)(i0 + c) * N + j] = x[c];
      for (int r = 0; r < i0; ++r) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c < nbw) s += P[c * ldp + r] * x[c];
        G[(long)r * N + j] -= s;
      }
    }
    __syncthreads();
  }
}

static size_t finish_lds(int N, int nb) {
  size_t panel = sizeof(double) * (size_t)nb * N;
  const size_t tile = sizeof(double) * 32 * 33;
  if (panel < tile) panel = tile;
  return panel + sizeof(double) * FN_WAVES + sizeof(int) * (FN_WAVES + 2);
}

int launch_finish(Plan& p, int batch, const UdvRef& f, double* G, double* logabs, int8_t* sign, int32_t* status,
                  hipStream_t st) {
  FinishArgs a;
  a.N = p.n;
  a.U = f.U;
  a.D = f.D;
  a.V = f.V;
  a.nref = f.nref;
  a.W = p.W;
  a.ipiv = p.ipiv;
  a.G = G;
  a.logabs = logabs;
  a.sign = sign;
  a.status = status;
  const int nb = p.n <= 1024 ? 16 : 8;
  const size_t lds = finish_lds(p.n, nb);
  if (nb == 16) {
    allow_max_lds((const void*)k_finish<16>);
    k_finish<16><<<batch, FN_THREADS, lds, st>>>(a);
  } else {
    allow_max_lds((const void*)k_finish<8>);
    k_finish<8><<<batch, FN_THREADS, lds, st>>>(a);
  }
  SLQ_LAUNCHED();
  return SLQ_OK;
}

}  // namespace slq
