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
// with partial pivoting (blocked: the panel is factored in LDS, its row
// interchanges are applied to the other columns as one gather, and the
// trailing update runs over (column, 16-row) work items so that every thread
// keeps a block of loads in flight).
#include "slq_internal.h"
#include "lu_interchange.h"

namespace slq {

constexpr int FN_THREADS = 512;
constexpr int FN_WAVES = FN_THREADS / 64;
constexpr int FN_RB = 8;            // rows per work item of the rank-NB updates
constexpr int FN_TS = 32;           // transpose tile: FN_TS source columns
constexpr int FN_TW = 4 * FN_TS;    // ... by FN_TW source rows

struct FinishArgs {
  int N;
  const double* U;
  const double* D;
  const double* V;
  const int32_t* nref;
  double* W;
  double* G;  // may be null
  double* logabs;
  int8_t* sign;
  int32_t* status;
};

// out[orow[k]][j] = src[j][k] / max(D[k], 1)  (+ min(D[k], 1) addm[k][j] when
// addm != null; orow null is the identity), through LDS tiles of FN_TS source
// columns by FN_TW source rows: coalesced on both sides.
__device__ void transpose_scaled(int N, const double* __restrict__ src, const double* __restrict__ D,
                                 const double* __restrict__ addm, double* __restrict__ out, double* tile,
                                 const uint16_t* orow) {
  constexpr int PER = FN_TS * FN_TW / FN_THREADS;
  const int nk = (N + FN_TS - 1) / FN_TS, nj = (N + FN_TW - 1) / FN_TW;
  for (int t = 0; t < nk * nj; ++t) {
    const int k0 = (t / nj) * FN_TS, jb = (t % nj) * FN_TW;
    double v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * FN_THREADS;
      const int j = jb + e / FN_TS, k = k0 + e % FN_TS;  // source row j, column k
      v[q] = (j < N && k < N) ? src[(long)j * N + k] : 0.0;
    }
    __syncthreads();  // the previous tile has been read
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * FN_THREADS;
      tile[(e / FN_TS) * (FN_TS + 1) + e % FN_TS] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * FN_THREADS;
      const int kk = e / FN_TW, jj = e % FN_TW;
      const int k = k0 + kk, j = jb + jj;
      if (k < N && j < N) {
        const double d = D[k];
        double x = tile[jj * (FN_TS + 1) + kk] / fmax(d, 1.0);
        if (addm) x += fmin(d, 1.0) * addm[(long)k * N + j];
        out[(long)(orow ? orow[k] : k) * N + j] = x;
      }
    }
  }
  __syncthreads();
}

// A[rowoff + r][j] -= sum_c P[c][r] A[xrow0 + c][j] for r in [rbeg, rend), j in
// [jbeg, jend): the rank-nbw update of LU and of the two triangular solves.
// Work items are (column, FN_RB consecutive rows), columns fastest, so that
// a thread has FN_RB + NB loads in flight at once and the rows of a wave are
// coalesced.  The rows xrow0.. are disjoint from the updated ones.
// Where N, ldp, rbeg and jbeg are even, an item is a pair of adjacent columns
// and 4 rows instead: 16-byte loads and stores, and each 16-byte read of P
// serves two rows of both columns.
template <int NB>
__device__ __forceinline__ void rank_update(double* __restrict__ A, int N, const double* P, int ldp, int nbw,
                                            int xrow0, int rowoff, int rbeg, int rend, int jbeg, int jend) {
  const int ncol = jend - jbeg;
  if (ncol <= 0 || rend <= rbeg) return;
  if (((N | ldp | rbeg | jbeg) & 1) == 0) {
    typedef double d2_t __attribute__((ext_vector_type(2)));
    const int npair = ncol / 2;  // ncol = N - jbeg is even too
    constexpr int RB2 = 4;  // rows per item: x and w of two columns stay in registers
    const int nch = (rend - rbeg + RB2 - 1) / RB2;
    for (int it = threadIdx.x; it < npair * nch; it += FN_THREADS) {
      const int j = jbeg + 2 * (it % npair);
      const int r0 = rbeg + (it / npair) * RB2;
      d2_t w[RB2], acc[RB2];
#pragma unroll
      for (int q = 0; q < RB2; ++q) {
        w[q] = r0 + q < rend ? *(const d2_t*)(A + (long)(rowoff + r0 + q) * N + j) : d2_t{0.0, 0.0};
        acc[q] = d2_t{0.0, 0.0};
      }
      constexpr int CH = NB < 8 ? NB : 8;  // columns of P per pass (registers)
#pragma unroll
      for (int c0 = 0; c0 < NB; c0 += CH) {
        d2_t x[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c)
          x[c] = c0 + c < nbw ? *(const d2_t*)(A + (long)(xrow0 + c0 + c) * N + j) : d2_t{0.0, 0.0};
#pragma unroll
        for (int q2 = 0; q2 < RB2; q2 += 2)
#pragma unroll
          for (int c = 0; c < CH; ++c)
            if (c0 + c < nbw && r0 + q2 < rend) {
              const d2_t pc = *(const d2_t*)(P + (c0 + c) * ldp + r0 + q2);  // rows r0+q2, r0+q2+1
              acc[q2] += pc[0] * x[c];
              acc[q2 + 1] += pc[1] * x[c];
            }
      }
#pragma unroll
      for (int q = 0; q < RB2; ++q) w[q] -= acc[q];
#pragma unroll
      for (int q = 0; q < RB2; ++q)
        if (r0 + q < rend) *(d2_t*)(A + (long)(rowoff + r0 + q) * N + j) = w[q];
    }
    return;
  }
  const int nch = (rend - rbeg + FN_RB - 1) / FN_RB;
  for (int it = threadIdx.x; it < ncol * nch; it += FN_THREADS) {
    const int j = jbeg + it % ncol;
    const int r0 = rbeg + (it / ncol) * FN_RB;
    double x[NB], w[FN_RB];
#pragma unroll
    for (int c = 0; c < NB; ++c) x[c] = c < nbw ? A[(long)(xrow0 + c) * N + j] : 0.0;
#pragma unroll
    for (int q = 0; q < FN_RB; ++q) w[q] = r0 + q < rend ? A[(long)(rowoff + r0 + q) * N + j] : 0.0;
#pragma unroll
    for (int q = 0; q < FN_RB; ++q) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nbw && r0 + q < rend) s += P[c * ldp + r0 + q] * x[c];
      w[q] -= s;
    }
#pragma unroll
    for (int q = 0; q < FN_RB; ++q)
      if (r0 + q < rend) A[(long)(rowoff + r0 + q) * N + j] = w[q];
  }
}

template <int NB>
__global__ __launch_bounds__(FN_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_finish(FinishArgs a) {
  extern __shared__ double lds[];
  const int N = a.N;
  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long NN = (long)N * N;
  const double* U = a.U + b * NN;
  const double* V = a.V + b * NN;
  const double* D = a.D + (long)b * N;
  double* W = a.W + b * NN;

  const int ldp = N;
  double* P = lds;                                           // [NB][N] panel, or the transpose tile
  double* redv = P + max(NB * N, FN_TW * (FN_TS + 1));       // [FN_WAVES]
  int* redi = (int*)(redv + FN_WAVES);                       // [FN_WAVES]
  int* flag = redi + FN_WAVES;                               // [2] a zero pivot / a refused pivot index
  int* nsl = flag + 2;                                       // [1] rows touched by a panel's interchanges
  int* srow = nsl + 1;                                       // [2 NB] those rows, the panel's own first
  int* ssrc = srow + 2 * NB;                                 // [2 NB] row whose entries each one receives
  uint16_t* ipiv = (uint16_t*)(ssrc + 2 * NB);               // [N] pivot rows
  uint16_t* orow = ipiv + N;                                 // [N] row permutation of the solves
  if (tid == 0) flag[0] = flag[1] = 0;

  // ---- M = D_b^{-1} U^T + D_s V
  transpose_scaled(N, U, D, V, W, P, nullptr);

  // ---- LU with partial pivoting, in place, panels of NB columns
  for (int j0 = 0; j0 < N; j0 += NB) {
    const int nbw = min(NB, N - j0);
    const int m = N - j0;
    for (int idx = tid; idx < m * nbw; idx += FN_THREADS) {
      const int c = idx % nbw, r = idx / nbw;
      P[c * ldp + r] = W[(long)(j0 + r) * N + j0 + c];
    }
    __syncthreads();
    {  // largest entry of the panel's first column
      double cb = -1.0;
      int ci = m;
      for (int r = tid; r < m; r += FN_THREADS) {
        const double v = fabs(P[r]);
        if (v > cb) {
          cb = v;
          ci = r;
        }
      }
      wave_argmax(cb, ci);
      if (lane == 0) {
        redv[wave] = cb;
        redi[wave] = ci;
      }
    }
    __syncthreads();
    for (int c = 0; c < nbw; ++c) {
      double best = redv[0];
      int bi = redi[0];
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
      __syncthreads();  // pivot row in place; the wave maxima have been read
      // multipliers of column c, update of the panel's later columns, and the
      // largest entry of column c + 1, row by row
      const double inv = zero ? 0.0 : 1.0 / P[c * ldp + c];
      double cb = -1.0;
      int ci = m;
      for (int r = c + 1 + tid; r < m; r += FN_THREADS) {
        if (!zero) {
          const double l = P[c * ldp + r] * inv;
          P[c * ldp + r] = l;
          for (int c2 = c + 1; c2 < nbw; ++c2) P[c2 * ldp + r] -= l * P[c2 * ldp + c];
        }
        if (c + 1 < nbw) {
          const double v = fabs(P[(c + 1) * ldp + r]);
          if (v > cb) {
            cb = v;
            ci = r;
          }
        }
      }
      wave_argmax(cb, ci);
      if (lane == 0) {
        redv[wave] = cb;
        redi[wave] = ci;
      }
      __syncthreads();
    }
    for (int idx = tid; idx < m * nbw; idx += FN_THREADS) {
      const int c = idx % nbw, r = idx / nbw;
      W[(long)(j0 + r) * N + j0 + c] = P[c * ldp + r];
    }
    // the panel's row interchanges as one permutation of the rows they touch
    // (a pivot outside the rows below the diagonal is refused and reported)
    if (tid == 0) {
      int ns = 0;
      if (lu_panel_permutation(N, j0, nbw, ipiv, srow, ssrc, &ns)) flag[1] = 1;
      nsl[0] = ns;
    }
    __syncthreads();
    // columns outside the panel: interchanges (all loads before any store),
    // then U12 = L11^{-1} A12 on the right
    const int ns = nsl[0];
    for (int j = tid; j < N; j += FN_THREADS) {
      if (j >= j0 && j < j0 + nbw) continue;
      double o[2 * NB];
#pragma unroll
      for (int k = 0; k < 2 * NB; ++k) o[k] = k < ns ? W[(long)ssrc[k] * N + j] : 0.0;
#pragma unroll
      for (int k = 0; k < 2 * NB; ++k)
        if (k >= nbw && k < ns) W[(long)srow[k] * N + j] = o[k];
      if (j >= j0 + nbw) {
#pragma unroll
        for (int c = 1; c < NB; ++c)
          if (c < nbw) {
#pragma unroll
            for (int c2 = 0; c2 < c; ++c2) o[c] -= P[c2 * ldp + c] * o[c2];
          }
      }
#pragma unroll
      for (int k = 0; k < NB; ++k)
        if (k < nbw) W[(long)(j0 + k) * N + j] = o[k];
    }
    __syncthreads();
    // trailing update A22 -= L21 U12
    rank_update<NB>(W, N, P, ldp, nbw, j0, j0, nbw, m, j0 + nbw, N);
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
    if (flag[1] && a.status) a.status[b] |= SLQ_ST_PIVOT;
    if (!isfinite(tot) && !sing && a.status) a.status[b] |= SLQ_ST_NONFINITE;
    a.logabs[b] = sing ? -INFINITY : tot;
    a.sign[b] = sing ? 0 : (pp ? -1 : 1);
  }
  if (!a.G) return;

  // ---- G = M^{-1} D_b^{-1} U^T: the LU's row interchanges, applied in order,
  // move row k of the right-hand side to row orow[k]
  if (tid == 0) {
    for (int k = 0; k < N; ++k) orow[k] = k;  // first: the source row of each position
    for (int k = 0; k < N; ++k) {
      const int pr = ipiv[k];
      if (pr != k) {
        const uint16_t t = orow[k];
        orow[k] = orow[pr];
        orow[pr] = t;
      }
    }
  }
  __syncthreads();
  for (int k = tid; k < N; k += FN_THREADS) ipiv[orow[k]] = k;  // inverted, into the free pivot array
  __syncthreads();
  double* G = a.G + b * NN;
  transpose_scaled(N, U, D, nullptr, G, P, ipiv);
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
        if (c < nbw) {
#pragma unroll
          for (int c2 = 0; c2 < c; ++c2) x[c] -= P[c2 * ldp + c] * x[c2];
        }
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nbw) G[(long)(i0 + c) * N + j] = x[c];
    }
    __syncthreads();
    rank_update<NB>(G, N, P, ldp, nbw, i0, i0, nbw, m, 0, N);
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
#pragma unroll
          for (int c2 = c + 1; c2 < NB; ++c2)
            if (c2 < nbw) s -= P[c2 * ldp + i0 + c] * x[c2];
          x[c] = s / P[c * ldp + i0 + c];
        }
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nbw) G[(long)(i0 + c) * N + j] = x[c];
    }
    __syncthreads();
    rank_update<NB>(G, N, P, ldp, nbw, i0, 0, 0, i0, 0, N);
    __syncthreads();
  }
}

static size_t finish_lds(int N, int nb) {
  size_t panel = (size_t)nb * N;
  if (panel < (size_t)FN_TW * (FN_TS + 1)) panel = (size_t)FN_TW * (FN_TS + 1);
  return sizeof(double) * (panel + FN_WAVES) + sizeof(int) * (FN_WAVES + 3 + 4 * nb) + sizeof(uint16_t) * 2 * N;
}

int launch_finish(Plan& p, int batch, const UdvRef& f, double* G, double* logabs, int8_t* sign, int32_t* status,
                  hipStream_t st) {
  // without G the determinant comes from a QR of M on the matrix cores
  // ((4/3) N^3 flops per field for R), with G from an LU ((2/3) N^3) and the
  // two triangular solves (2 N^3)
  const double n3 = (double)p.n * p.n * p.n;
  if (!G && use_det_qr(p, f))
    return timed_part(p, SLQ_PROFILE_FINISH, batch * 4.0 / 3.0 * n3, st,
                      [&]() { return launch_det_qr(p, batch, f, logabs, sign, status, st); });
  return timed_part(p, SLQ_PROFILE_FINISH, batch * (G ? 8.0 / 3.0 : 2.0 / 3.0) * n3, st,
                    [&]() { return launch_finish_lu(p, batch, f, G, logabs, sign, status, st); });
}

int launch_finish_lu(Plan& p, int batch, const UdvRef& f, double* G, double* logabs, int8_t* sign, int32_t* status,
                     hipStream_t st) {
  FinishArgs a;
  a.N = p.n;
  a.U = f.U;
  a.D = f.D;
  a.V = f.V;
  a.nref = f.nref;
  a.W = p.W;
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
