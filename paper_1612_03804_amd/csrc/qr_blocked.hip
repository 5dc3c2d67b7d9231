// Blocked Householder QR of a batch of pre-pivoted matrices, MFMA trailing
// updates (the stabilisation step of the slice-matrix chain; see qr.hip for
// the factorisation that is computed and why).
//
// For each panel of NB columns:
//   k_panel   one workgroup per field factors the m x NB panel in registers
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
// ties); W[:, c] = X[:, perm[c]] * D[perm[c]].  With norm2 (the squared
// column norms of X, from the kernel that produced it) X is read once; a
// column whose plain sum of squares over- or underflowed is summed again here
// with rescaling.
__global__ __launch_bounds__(PQ_THREADS) void k_prepivot(int N, const double* __restrict__ Xall,
                                                         double* __restrict__ Wall, const double* __restrict__ Dall,
                                                         int32_t* __restrict__ permall, int32_t* status,
                                                         const double* __restrict__ norm2all) {
  extern __shared__ double lds[];
  const int b = blockIdx.x;
  const long NN = (long)N * N;
  const double* X = Xall + b * NN;
  double* W = Wall + b * NN;
  const double* D = Dall + (long)b * N;
  int32_t* perm = permall + (long)b * N;
  double* nrm = lds;           // [N] scaled column norms, then the scale of the c-th pivoted column
  int* rp = (int*)(lds + N);   // [N]
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int j = threadIdx.x; j < N; j += PQ_THREADS) {
    double ss = 0.0, mx = 0.0;
    if (norm2all) {
      ss = norm2all[(long)b * N + j];
      mx = ss > 0.0 ? 1.0 : 0.0;  // the rescaled pass below finds the true maximum if it is needed
    } else {
#pragma unroll 8
      for (int i = 0; i < N; ++i) {
        const double v = X[(long)i * N + j];
        ss += v * v;
        mx = fmax(mx, fabs(v));
      }
    }
    double nv = sqrt(ss);
    if (!(nv < INFINITY) || (nv < 1e-150 && mx > 0.0)) {  // rescale when the plain sum over/underflows
      if (norm2all) {
        mx = 0.0;
        for (int i = 0; i < N; ++i) mx = fmax(mx, fabs(X[(long)i * N + j]));
      }
      ss = 0.0;
      const double inv = 1.0 / mx;
#pragma unroll 8
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
#pragma unroll 8
    for (int i = 0; i < N; ++i) {
      const double ni = nrm[i];
      r += (ni > nj) || (ni == nj && i < j);
    }
    rp[r] = j;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < N; c += PQ_THREADS) {
    perm[c] = rp[c];
    nrm[c] = D[rp[c]];
  }
  __syncthreads();
  // W[:, c] = X[:, perm[c]] D[perm[c]]: one wave per row, lanes along the row;
  // the loads of two rows, up to 512 columns each, are in flight together
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int CU = 8;  // columns per lane and row in flight
  for (int c0 = 0; c0 < N; c0 += 64 * CU) {
    for (int i = wave; i < N; i += 2 * PQ_WAVES) {
      const int i2 = i + PQ_WAVES;
      const double* xr = X + (long)i * N;
      const double* xr2 = X + (long)i2 * N;
      double v[CU], v2[CU];
#pragma unroll
      for (int u = 0; u < CU; ++u) {
        const int c = c0 + lane + 64 * u;
        const bool in = c < N;
        v[u] = in ? xr[rp[c]] : 0.0;
        v2[u] = in && i2 < N ? xr2[rp[c]] : 0.0;
      }
      double* wr = W + (long)i * N;
      double* wr2 = W + (long)i2 * N;
#pragma unroll
      for (int u = 0; u < CU; ++u) {
        const int c = c0 + lane + 64 * u;
        if (c < N) {
          wr[c] = v[u] * nrm[c];
          if (i2 < N) wr2[c] = v2[u] * nrm[c];
        }
      }
    }
  }
  if (threadIdx.x == 0 && bad && status) atomicOr(&status[b], SLQ_ST_NONFINITE);
}

// --------------------------------------------------------------- panel ----
// Sums over the wave of 2 or 4 values at once.  The lane-swap instructions of
// gfx950 fold the halves and then the 16-lane rows of two values into one
// register (permlane32_swap exchanges the upper 32 lanes of its first operand
// with the lower 32 of its second, permlane16_swap the odd rows of the first
// with the even rows of the second), so that each row holds one value's
// partial sums; DPP moves finish the rows.  Every lane returns the same sums.
__device__ __forceinline__ double pq_fold32(double x, double y) {
  // lanes 0-31: x[l] + x[l + 32]; lanes 32-63: y[l - 32] + y[l]
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(x), (unsigned)__double2loint(y), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(x), (unsigned)__double2hiint(y), false, false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ double pq_fold16(double x, double y) {
  // rows 0 and 2: x's rows (0, 1) and (2, 3) summed; rows 1 and 3: y's
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(x), (unsigned)__double2loint(y), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(x), (unsigned)__double2hiint(y), false, false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ double pq_row_sum(double v) {
  v += dpp_move<DPP_QUAD_XOR1>(v);
  v += dpp_move<DPP_QUAD_XOR2>(v);
  v += dpp_move<DPP_ROW_ROR4>(v);
  return v + dpp_move<DPP_ROW_ROR8>(v);
}
template <int C>
__device__ __forceinline__ void pq_wave_sums(double (&s)[C]) {
  static_assert(C == 1 || C == 2 || C == 4, "2 or 4 values, or one");
  if constexpr (C == 1) {
    s[0] = wave_sum(s[0]);
  } else if constexpr (C == 2) {
    const double r = pq_row_sum(pq_fold16(pq_fold32(s[0], s[1]), pq_fold32(s[0], s[1])));
    s[0] = read_lane(r, 0);   // rows 0, 1
    s[1] = read_lane(r, 32);  // rows 2, 3
  } else {
    const double r = pq_row_sum(pq_fold16(pq_fold32(s[0], s[2]), pq_fold32(s[1], s[3])));
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q] = read_lane(r, 16 * q);  // row q
  }
}

struct PanelArgs {
  int N, j0, nbw;
  double* W;       // [b][N][N]: panel columns j0..j0+nbw, rows j0..N-1 (in: A, out: R above / V below)
  double* Vbuf;    // [b][N][N]: explicit V of the panel at rows zrow0.., columns j0..j0+nbw
  int zrow0;       // rows zrow0..j0-1 of V are written as zeros
  double* T;       // [b] + strideT: compact-WY factor of this panel, row stride ldt
  long strideT;
  int ldt, tzero;  // rows nbw..tzero-1 of the panel's T columns are written as zeros
  double* D;       // [b][N] out: |R_jj|
  double* invD;    // [b][N] out: 1/|R_jj|
  int32_t* nref;   // [b] in/out: reflectors with tau != 0
  int32_t* status;
};

// One workgroup per field factors the m x nbw panel.  Wave w owns the
// columns c = w (mod waves) and keeps them in registers, row r = lane + 64 k
// in slot k (RPL slots cover m); the panel comes in and goes out 64 rows at
// a time through a small LDS chunk, so that several fields share a CU.  Step
// c: the owner of column c has formed reflector c (LAPACK dlarfg: beta =
// -sign(alpha) ||x||, v = x / (alpha - beta) below the diagonal) and
// published v_c in LDS; after one barrier every wave applies H_c = I - tau_c
// v_c v_c^T to its own columns > c (the owner of column c+1 first, and it
// forms and publishes reflector c+1 at once, into the other of two buffers)
// and adds the Gram entries v_i . v_c of its finished columns i < c.  T
// (Q_panel = I - V T V^T) follows from the Gram matrix at the end.
template <int NB, int RPL, bool CACHE_V, int TH>
__global__ __launch_bounds__(TH) __attribute__((amdgpu_waves_per_eu(TH == 1024 ? 4 : (NB == 32 ? 4 : 1)))) void k_panel(PanelArgs a) {
  constexpr int PQ_THREADS = TH, PQ_WAVES = TH / 64;
  extern __shared__ double lds[];
  constexpr int CPW = NB >= PQ_WAVES ? NB / PQ_WAVES : 1;  // columns per wave
  constexpr int LT = NB + 1;                 // padded row stride of T and the Gram matrix
  constexpr int LS = 65;                     // padded column stride of the 64-row chunk
  constexpr int VR = 64 * RPL;               // length of a published reflector
  constexpr int SPT = 64 * NB / PQ_THREADS;  // chunk entries per thread
  static_assert(SPT * PQ_THREADS == 64 * NB, "a chunk is 64 rows of NB columns");
  const int N = a.N, j0 = a.j0, nbw = a.nbw, m = N - j0;
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long NN = (long)N * N;
  const int nch = (m + 63) / 64;    // chunks that hold rows (<= RPL)
  double* W = a.W + b * NN;
  double* S = lds;                  // [NB][LS]: 64 rows of the panel on their way in or out
  double* Vp = S + NB * LS;         // [2][VR]: the reflectors of two consecutive steps
  double* T = Vp + 2 * VR;          // [NB][LT]
  double* Gm = T + NB * LT;         // [NB][LT]
  double* tau = Gm + NB * LT;       // [NB]

  // panel -> registers: row-wise (coalesced) reads, transposed through S;
  // the next chunk's reads are in flight while a chunk is distributed
  double col[CPW][RPL];
  double stg[SPT];
  auto chunk_load = [&](int k) {
#pragma unroll
    for (int t = 0; t < SPT; ++t) {
      const int e = tid + t * PQ_THREADS;
      const int i = e / NB, c = e % NB, r = 64 * k + i;
      stg[t] = (c < nbw && r < m) ? W[(long)(j0 + r) * N + j0 + c] : 0.0;
    }
  };
  chunk_load(0);
#pragma unroll
  for (int k = 0; k < RPL; ++k) {
    if (k < nch) {
      __syncthreads();  // S is free
#pragma unroll
      for (int t = 0; t < SPT; ++t) {
        const int e = tid + t * PQ_THREADS;
        S[(e % NB) * LS + e / NB] = stg[t];
      }
      __syncthreads();
      if (k + 1 < nch) chunk_load(k + 1);
#pragma unroll
      for (int q = 0; q < CPW; ++q) col[q][k] = S[(wave + PQ_WAVES * q) * LS + lane];
    } else {
#pragma unroll
      for (int q = 0; q < CPW; ++q) col[q][k] = 0.0;
    }
  }

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
    double* vp = Vp + (c & 1) * VR;
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
      const int r = lane + 64 * k;
      if (r == c) col[q][k] = beta;
      if (r > c && r < m) vp[r] = col[q][k];
    }
    if (lane == 0) tau[c] = tc;
  };

  if (wave == 0) reflect(0, 0);
  for (int c = 0; c < nbw; ++c) {
    __syncthreads();  // reflector c is published; step c - 1 is done everywhere
    const double tc = tau[c];
    const double* vp = Vp + (c & 1) * VR;
    double vr[CACHE_V ? RPL : 1];
    auto vrow = [&](int k) -> double {  // v_c at row lane + 64 k
      const int r = lane + 64 * k;
      return r < c || r >= m ? 0.0 : (r == c ? 1.0 : vp[r]);
    };
    if (CACHE_V) {
#pragma unroll
      for (int k = 0; k < RPL; ++k) vr[k] = vrow(k);
    }
    // the dot products v_c . col of the owned columns, reduced together
    double s[CPW];
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < RPL; ++k) t += (CACHE_V ? vr[k] : vrow(k)) * col[q][k];
      s[q] = t;
    }
    pq_wave_sums<CPW>(s);
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      const int c2 = wave + PQ_WAVES * q;
      if (c2 >= nbw) continue;
      if (c2 > c) {  // apply H_c
        if (tc != 0.0) {
          const double st = s[q] * tc;
#pragma unroll
          for (int k = 0; k < RPL; ++k) col[q][k] -= st * (CACHE_V ? vr[k] : vrow(k));
        }
        if (c2 == c + 1) reflect(q, c2);
      } else if (c2 < c) {  // finished column: Gram entry v_{c2} . v_c
        if (lane == 0) Gm[c2 * LT + c] = s[q];
      }
    }
  }
  // (the first barrier of the write-back also orders the last step and the
  // Gram entries before the T build that follows it)
  // registers -> R (on and above the diagonal) and V (below) in W, explicit V
  // (unit diagonal, zeros above) in Vbuf, 64 rows at a time through S
  double* Vb = a.Vbuf + b * NN;
#pragma unroll
  for (int k = 0; k < RPL; ++k) {
    if (k < nch) {
      __syncthreads();  // S is free
#pragma unroll
      for (int q = 0; q < CPW; ++q) S[(wave + PQ_WAVES * q) * LS + lane] = col[q][k];
      __syncthreads();
      if (k == 0 && wave == 0) {  // |R_jj| of the panel's columns
        const bool live = lane < nbw;
        const double d = live ? fabs(S[lane * LS + lane]) : 1.0;
        const unsigned long long bad = __ballot(live && (!(d > 0.0) || !(d < INFINITY)));
        if (live) {
          a.D[(long)b * N + j0 + lane] = d;
          a.invD[(long)b * N + j0 + lane] = 1.0 / d;
        }
        if (lane == 0 && bad && a.status) atomicOr(&a.status[b], SLQ_ST_NONFINITE);
      }
#pragma unroll
      for (int t = 0; t < SPT; ++t) {
        const int e = tid + t * PQ_THREADS;
        const int i = e / NB, c = e % NB, r = 64 * k + i;
        if (c < nbw && r < m) {
          const double pv = S[c * LS + i];
          W[(long)(j0 + r) * N + j0 + c] = pv;
          Vb[(long)(j0 + r) * N + j0 + c] = (r == c) ? 1.0 : (r > c ? pv : 0.0);
        }
      }
    }
  }
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
    const unsigned long long refl = __ballot(live && tau[lane] != 0.0);
    if (lane == 0) a.nref[b] += __popcll(refl);
  }
  __syncthreads();  // T is in LDS
  for (int r = a.zrow0 + tid / NB; r < j0; r += PQ_THREADS / NB) {
    const int c = tid % NB;
    if (c < nbw) Vb[(long)r * N + j0 + c] = 0.0;
  }
  double* Tg = a.T + b * a.strideT;
  for (int idx = tid; idx < a.tzero * NB; idx += PQ_THREADS) {
    const int i = idx / NB, j = idx % NB;
    if (j < nbw) Tg[(long)i * a.ldt + j] = i < nbw ? T[i * LT + j] : 0.0;
  }
}

// panel width and register rows per lane by matrix size: the widest panel
// whose columns fit the registers of one workgroup (RPL rows per lane and
// column, 64 * RPL >= N)
template <int NB, int RPL>
struct PanelShape {
  static constexpr bool CACHE = RPL <= 18;  // keep the published reflector in registers too
};

// Compact-WY factor of a whole outer block, Q_O = Q_1 ... Q_P = I - V_O T_O V_O^T,
// from the panels' own factors T_p (on T_O's diagonal, written by k_panel)
// and the Gram matrix S = V_O^T V_O of the block's reflectors:
//     T_O[0:s, P] = -T_O[0:s, 0:s] S[0:s, P] T_P,  s = first column of panel P,
// panel by panel (the usual recursive form of T_O = [[T_A, -T_A V_A^T V_B T_B],
// [0, T_B]]).  One workgroup per field; T_O is built in LDS and written back
// (blocks of at most QR_NBO columns).
constexpr int TB_THREADS = 256;
constexpr int TB_LT = QR_NBO + 1;  // padded row stride of T in LDS
constexpr int TB_CH = 8;           // columns of a panel per step

__global__ __launch_bounds__(TB_THREADS) void k_tbuild(int wo, int nb, double* __restrict__ TOall, long strideT, int ldt,
                                                       const double* __restrict__ Sall, long strideS, int lds_) {
  extern __shared__ double lds[];
  double* T = lds;                    // [QR_NBO][TB_LT]
  double* Y = T + QR_NBO * TB_LT;     // [QR_NBO][TB_CH]
  const long b = blockIdx.x;
  double* Tg = TOall + b * strideT;
  const double* S = Sall + b * strideS;
  const int tid = threadIdx.x;
  // the panels' diagonal blocks, zeros elsewhere
  for (int e = tid; e < wo * wo; e += TB_THREADS) {
    const int i = e / wo, j = e % wo;
    T[i * TB_LT + j] = (i / nb == j / nb && i <= j) ? Tg[(long)i * ldt + j] : 0.0;
  }
  __syncthreads();
  for (int s0 = nb; s0 < wo; s0 += nb) {
    const int nbw = min(nb, wo - s0);
    for (int c0 = 0; c0 < nbw; c0 += TB_CH) {
      const int nc = min(TB_CH, nbw - c0);
      // Y[k][c] = sum_d S[k][s0 + d] T[s0 + d][s0 + c0 + c], k < s0 (T_P upper triangular)
      for (int e = tid; e < s0 * nc; e += TB_THREADS) {
        const int k = e / nc, c = e % nc;
        double y = 0.0;
        for (int d = 0; d <= c0 + c; ++d) y += S[(long)k * lds_ + s0 + d] * T[(s0 + d) * TB_LT + s0 + c0 + c];
        Y[k * TB_CH + c] = y;
      }
      __syncthreads();
      // T[i][s0 + c0 + c] = -sum_{k = i}^{s0 - 1} T[i][k] Y[k][c]
      for (int e = tid; e < s0 * nc; e += TB_THREADS) {
        const int i = e % s0, c = e / s0;
        double t = 0.0;
        for (int k = i; k < s0; ++k) t += T[i * TB_LT + k] * Y[k * TB_CH + c];
        T[i * TB_LT + s0 + c0 + c] = -t;
      }
      __syncthreads();
    }
  }
  for (int e = tid; e < wo * wo; e += TB_THREADS) {
    const int i = e / wo, j = e % wo;
    Tg[(long)i * ldt + j] = T[i * TB_LT + j];
  }
}

__global__ void k_zero_i32(int32_t* x, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x[i] = 0;
}

// Blocking: panels of NB columns inside outer blocks of NBOT columns.  A
// panel's reflectors update the rest of its block at once; the trailing
// columns beyond the outer block, and later Q, are updated once per outer
// block with its combined compact-WY factor
//     T_O = [[T_A, -T_A (V_A^T V_B) T_B], [0, T_B]]
// so the large blocks are read and written once per NBOT columns.  When NBOT
// does not divide N the short block comes first: every later block then
// starts NBOT-aligned from the end, so the large updates have row and column
// counts that are multiples of the 128 x 64 tiles (N = 400: 384 x 256 and
// 256 x 128 instead of 400 x 272 and 272 x 144).
//
// With narrow panels (NB <= 8, large N) there are two more levels: mid
// blocks of NBM columns inside sub-blocks of at most QR_NBO columns inside the
// outer block.  A panel updates only the rest of its mid block; a mid block,
// with its factor T_mid, the rest of its sub-block (rank NBM); a sub-block,
// with T_sub, the rest of the outer block (rank QR_NBO); the outer block the
// trailing matrix (rank NBOT).  T_mid and T_sub come from the Gram matrix of
// their reflectors and the panels' T (k_tbuild); T_O of two sub-blocks from
// the formula above, with V_A^T V_B over the rows of V_B and two small
// products.  Each level reads and writes the columns to its right a quarter
// (half, for the outer level) as often as the level below would.
template <int NB, int RPL, int NBOT, int TH = PQ_THREADS>
static int run_blocked(Plan& p, int batch, const double* X, const UdvRef& o, int32_t* status, hipStream_t st,
                       const double* norm2, bool form_q) {
  static_assert(NBOT == QR_NBO || NBOT == 2 * QR_NBO, "an outer block holds one or two sub-blocks");
  const int N = p.n;
  const long NN = (long)N * N;
  const int nout = (N + NBOT - 1) / NBOT;
  double* Vbuf = (X == p.Xa) ? p.Xb : p.Xa;  // free once W holds the pivoted copy of X
  const long sW = qr_workspace_per_field(N);
  const long sT = (long)NBOT * NBOT;
  double* TO = p.qrws;                   // [b]: [nout][NBOT][NBOT] outer factors
  double* Gb = TO + nout * sT;           // [QR_NBO][QR_NBO] Gram blocks
  double* Wt = Gb + (long)QR_NBO * QR_NBO;  // [NBOT][N]
  double* Wt2 = Wt + (long)NBOT * N;     // [NBOT][N]
  const size_t lpp = sizeof(double) * N + sizeof(int) * N;
  allow_max_lds((const void*)k_prepivot);
  k_prepivot<<<batch, PQ_THREADS, lpp, st>>>(N, X, p.W, o.D, p.perm, status, norm2);
  SLQ_LAUNCHED();
  k_zero_i32<<<(batch + 255) / 256, 256, 0, st>>>(o.nref, batch);
  SLQ_LAUNCHED();
  constexpr bool GRAM_T = NB <= 8;  // narrow panels: block factors from Gram products (below)
  // tiles from a sweep of these shapes on MI355X (N = 400, 256 fields): 128 x 64
  // with 8 wavefronts wherever the output has 64 rows or more, 32 x 64 with K 16
  // for the thin products of the panels, 16 x 64 for those of a 16-column block.
  // With narrow panels (N = 2304) the thin products stage K 32 deep: 298.6
  // against 304.1 ms per stabilisation of 256 fields (at N = 400, 6.37 against
  // 6.32 ms: K 16 stays there)
  constexpr int THIN32 = GRAM_T ? GEMM_32x64_K32 : GEMM_32x64, THIN16 = GRAM_T ? GEMM_16x64_K32 : GEMM_16x64;
  auto gemm = [&](int M, int Nc, int K, const double* A, long lda, long sA, bool ta, const double* B, long ldb,
                  long sB, double* C, long ldc, long sC, double alpha, double beta, int c_ident = 0,
                  int c_zero_rows = 0) -> int {
    GemmArgs g{};
    g.c_ident = c_ident;
    g.c_zero_rows = c_zero_rows;
    // the transposed products (V^T A) and, with narrow panels (N = 2304), all
    // products with a long K take 128 x 128 tiles of 64 x 64 per wavefront (V^T A
    // at N = 2304: 0.82 against 0.75 of the FP64 peak; at N = 400 6.20 against
    // 6.25 ms per stabilisation); untransposed products with a short K (the
    // rank-k updates) take the 128 x 64 tiles, whose eight wavefronts per SIMD
    // hide a short K better (0.66 against 0.57), without bounds checks where the
    // shape allows (0.70)
    const bool big = ta || (GRAM_T && K > 256);
    g.cfg = M >= 64 ? (big ? GEMM_BIG : (ta ? GEMM_128x64 : GEMM_LEAN)) : (M <= 16 ? THIN16 : THIN32);
    g.M = M;
    g.N = Nc;
    g.K = K;
    g.A = A;
    g.lda = lda;
    g.strideA = sA;
    g.B = B;
    g.ldb = ldb;
    g.strideB = sB;
    g.C = C;
    g.ldc = ldc;
    g.strideC = sC;
    g.alpha = alpha;
    g.beta = beta;
    g.batch = batch;
    return launch_gemm(g, ta, false, st);
  };
  // B <- B - V op(T) (V^T B): V m x k (ld N), T k x k (ld NBOT), B m x n (ld N)
  auto apply = [&](const double* Vp, const double* Tp, int k, double* Bp, int m, int n, bool transT) -> int {
    int rc = gemm(k, n, m, Vp, N, NN, true, Bp, N, NN, Wt, N, sW, 1.0, 0.0);
    if (rc == SLQ_OK) rc = gemm(k, n, k, Tp, NBOT, sW, transT, Wt, N, sW, Wt2, N, sW, 1.0, 0.0);
    if (rc == SLQ_OK) rc = gemm(m, n, k, Vp, N, NN, false, Wt2, N, sW, Bp, N, NN, -1.0, 1.0);
    return rc;
  };
  // How a block's T grows panel by panel: with narrow panels (many per block)
  // from one Gram product V^T V and k_tbuild after the block's panels (at N =
  // 2304, 8-column panels: 36 ms per 64-field evaluation against 150 ms of
  // thin products), with wide ones by three small products per panel (at N =
  // 400, 32-column panels over 512 fields the one-workgroup-per-CU k_tbuild
  // takes 7.8 ms per evaluation, the products less)
  constexpr int NBM = 32;
  auto gram = [&](int w, int row0, const double* V0) -> int {  // Gb = V0^T V0 over rows row0..N-1
    GemmArgs gg{};
    gg.M = w;
    gg.N = w;
    gg.K = N - row0;
    gg.A = V0;
    gg.lda = N;
    gg.strideA = NN;
    gg.B = V0;
    gg.ldb = N;
    gg.strideB = NN;
    gg.C = Gb;
    gg.ldc = QR_NBO;
    gg.strideC = sW;
    gg.alpha = 1.0;
    gg.beta = 0.0;
    gg.batch = batch;
    gg.cfg = THIN32;
    return launch_gemm(gg, true, false, st);
  };
  auto tbuild = [&](int w, double* Tsub) -> int {  // w <= QR_NBO
    const size_t tl = sizeof(double) * ((size_t)QR_NBO * TB_LT + QR_NBO * TB_CH);
    allow_max_lds((const void*)k_tbuild);
    k_tbuild<<<batch, TB_THREADS, tl, st>>>(w, NB, Tsub, sW, NBOT, Gb, sW, QR_NBO);
    SLQ_LAUNCHED();
    return SLQ_OK;
  };
  // blocks of width `full` over [0, n), the short one (n mod full) first
  auto bstart = [](int n, int full, int k) { const int r = n % full; return r == 0 ? k * full : (k == 0 ? 0 : r + (k - 1) * full); };
  auto bwidth = [](int n, int full, int k) { const int r = n % full; return r == 0 ? full : (k == 0 ? r : full); };
  for (int ob = 0; ob < nout; ++ob) {
    const int J0 = bstart(N, NBOT, ob), wo = bwidth(N, NBOT, ob);
    double* Tb = TO + ob * sT;
    const int nsub = (wo + QR_NBO - 1) / QR_NBO;
    for (int sb = 0; sb < nsub; ++sb) {
      const int S0 = J0 + bstart(wo, QR_NBO, sb), ws = bwidth(wo, QR_NBO, sb);
      const int wmid = GRAM_T && ws > NBM ? NBM : ws;  // mid-block width (the whole sub-block: two levels)
      for (int jm0 = S0; jm0 < S0 + ws; jm0 += wmid) {
        const int wm = std::min(wmid, S0 + ws - jm0), sftm = jm0 - J0;
        for (int j0 = jm0; j0 < jm0 + wm; j0 += NB) {
          const int nbw = std::min(NB, jm0 + wm - j0), m = N - j0, sft = j0 - J0;
          double* Tp = Tb + (long)sft * NBOT + sft;
          PanelArgs a{N, j0, nbw, p.W, Vbuf, J0, Tp, sW, NBOT, wo - sft, o.D, p.invD, o.nref, status};
          const size_t lds = sizeof(double) * ((size_t)NB * 65 + 2 * 64 * RPL + 2 * NB * (NB + 1) + NB);
          constexpr bool CACHE = PanelShape<NB, RPL>::CACHE;
          allow_max_lds((const void*)k_panel<NB, RPL, CACHE, TH>);
          k_panel<NB, RPL, CACHE, TH><<<batch, TH, lds, st>>>(a);
          SLQ_LAUNCHED();
          const int nin = jm0 + wm - j0 - nbw;  // rest of the mid block
          if (nin > 0) SLQ_TRY(apply(Vbuf + (long)j0 * N + j0, Tp, nbw, p.W + (long)j0 * N + j0 + nbw, m, nin, true));
          const int sfs = j0 - S0;
          if (!GRAM_T && sfs > 0) {  // T_sub[0:sfs, sfs:sfs+nbw] = -T_sub[0:sfs, 0:sfs] (V_A^T V_B) T_B, rows j0.. only
            double* Ts = Tb + (long)(S0 - J0) * (NBOT + 1);
            SLQ_TRY(gemm(sfs, nbw, m, Vbuf + (long)j0 * N + S0, N, NN, true, Vbuf + (long)j0 * N + j0, N, NN, Gb,
                         QR_NBO, sW, 1.0, 0.0));
            SLQ_TRY(gemm(sfs, nbw, nbw, Gb, QR_NBO, sW, false, Tp, NBOT, sW, Wt2, N, sW, 1.0, 0.0));
            SLQ_TRY(gemm(sfs, nbw, sfs, Ts, NBOT, sW, false, Wt2, N, sW, Ts + sfs, NBOT, sW, -1.0, 0.0));
          }
        }
        const int rest = S0 + ws - jm0 - wm;  // columns of the sub-block after this mid block
        if (wm < ws && rest > 0) {
          double* Tm = Tb + (long)sftm * NBOT + sftm;
          const double* Vm = Vbuf + (long)jm0 * N + jm0;
          SLQ_TRY(gram(wm, jm0, Vm));
          SLQ_TRY(tbuild(wm, Tm));
          SLQ_TRY(apply(Vm, Tm, wm, p.W + (long)jm0 * N + jm0 + wm, N - jm0, rest, true));
        }
      }
      if (GRAM_T && ws > NB) {  // T_sub from its Gram matrix (rows S0.. of V_sub)
        SLQ_TRY(gram(ws, S0, Vbuf + (long)S0 * N + S0));
        SLQ_TRY(tbuild(ws, Tb + (long)(S0 - J0) * (NBOT + 1)));
      }
      const int rso = J0 + wo - S0 - ws;  // columns of the outer block after this sub-block
      if (rso > 0)
        SLQ_TRY(apply(Vbuf + (long)S0 * N + S0, Tb + (long)(S0 - J0) * (NBOT + 1), ws, p.W + (long)S0 * N + S0 + ws,
                      N - S0, rso, true));
    }
    if (nsub == 2) {  // T_O[0:wa, wa:wo] = -T_A (V_A^T V_B) T_B
      const int wa = bwidth(wo, QR_NBO, 0), wb = wo - wa, SB = J0 + wa;
      SLQ_TRY(gemm(wa, wb, N - SB, Vbuf + (long)SB * N + J0, N, NN, true, Vbuf + (long)SB * N + SB, N, NN, Gb, QR_NBO,
                   sW, 1.0, 0.0));
      SLQ_TRY(gemm(wa, wb, wb, Gb, QR_NBO, sW, false, Tb + (long)wa * (NBOT + 1), NBOT, sW, Wt2, N, sW, 1.0, 0.0));
      SLQ_TRY(gemm(wa, wb, wa, Tb, NBOT, sW, false, Wt2, N, sW, Tb + wa, NBOT, sW, -1.0, 0.0));
    }
    if (J0 + wo < N)
      SLQ_TRY(apply(Vbuf + (long)J0 * N + J0, Tb, wo, p.W + (long)J0 * N + J0 + wo, N - J0, N - J0 - wo, true));
  }
  if (!form_q) return SLQ_OK;
  // explicit Q, backwards: U[J0:, J0:] <- Q_O U[J0:, J0:] = U - V_O (T_O (V_O^T U)),
  // starting from U = I.  Columns J0..J0+wo-1 of U still hold [I; 0] there (later
  // blocks only touch columns beyond), so for them V_O^T U = V_top^T, the unit
  // lower triangle of V_O: U[:, block] = [I; 0] - V_O (T_O V_top^T), one small and
  // one rank-wo GEMM.  U is never set to I in memory: the later blocks have
  // written U[J0+wo:, J0+wo:], the rank-wo GEMMs read the rest of their C as the
  // identity's entries (zeros in rows J0..J0+wo-1 beyond the block, I on it).
  for (int ob = nout - 1; ob >= 0; --ob) {
    const int J0 = bstart(N, NBOT, ob), wo = bwidth(N, NBOT, ob), m = N - J0;
    const double* Vp = Vbuf + (long)J0 * N + J0;
    double* Ub = o.U + (long)J0 * N + J0;
    if (m > wo) {  // columns beyond the block: their rows J0..J0+wo-1 are still zero
      const int n2 = m - wo;
      SLQ_TRY(gemm(wo, n2, n2, Vp + (long)wo * N, N, NN, true, Ub + (long)wo * N + wo, N, NN, Wt, N, sW, 1.0, 0.0));
      SLQ_TRY(gemm(wo, n2, wo, TO + ob * sT, NBOT, sW, false, Wt, N, sW, Wt2, N, sW, 1.0, 0.0));
      SLQ_TRY(gemm(m, n2, wo, Vp, N, NN, false, Wt2, N, sW, Ub + wo, N, NN, -1.0, 1.0, 0, wo));
    }
    GemmArgs y{};  // Wt2 = T_O V_top^T
    y.M = wo;
    y.N = wo;
    y.K = wo;
    y.A = TO + ob * sT;
    y.lda = NBOT;
    y.strideA = sW;
    y.B = Vp;
    y.ldb = N;
    y.strideB = NN;
    y.C = Wt2;
    y.ldc = N;
    y.strideC = sW;
    y.alpha = 1.0;
    y.batch = batch;
    y.cfg = THIN32;
    SLQ_TRY(launch_gemm(y, false, true, st));
    SLQ_TRY(gemm(m, wo, wo, Vp, N, NN, false, Wt2, N, sW, Ub, N, NN, -1.0, 1.0, 1));
  }
  return SLQ_OK;
}

// Outer block width by matrix size: two sub-blocks of QR_NBO columns where the
// panels are narrow (N = 2304, 256 fields: the rank-256 trailing and Q
// updates read and write the large blocks half as often as rank-128 ones)
static int qr_outer_width(int N) { return N > 1152 ? 2 * QR_NBO : QR_NBO; }

long qr_workspace_per_field(int N) {
  const long nbo = qr_outer_width(N);
  const long nout = (N + nbo - 1) / nbo;
  return nout * nbo * nbo + (long)QR_NBO * QR_NBO + 2L * nbo * N;
}

int launch_qr_blocked(Plan& p, int batch, const double* X, const UdvRef& o, int32_t* status, hipStream_t st,
                      const double* norm2, bool form_q) {
  if (p.n <= 448) return run_blocked<32, 7, QR_NBO>(p, batch, X, o, status, st, norm2, form_q);
  if (p.n <= 1152) return run_blocked<16, 18, QR_NBO>(p, batch, X, o, status, st, norm2, form_q);
  // (16 columns at 38 rows per lane spill registers both as two columns per
  // wave of 512 threads and as one per wave of 1024)
  return run_blocked<8, 38, 2 * QR_NBO>(p, batch, X, o, status, st, norm2, form_q);
}

}  // namespace slq
