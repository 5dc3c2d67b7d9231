// Batched FP64 GEMM on the CDNA4 matrix cores (v_mfma_f64_16x16x4_f64).
//
//   C[b] = alpha * diag(rowscale_b) * op(A[b]) * diag(r_b) * op(B[b]) + beta * C[b]
//
// r_b is the field factor of one slice, exp(-+dtau xi s_{k,l}) ("Basics of
// DQMC": B_l = exp(-dtau K) exp(V(s_l))), applied to the rows of op(B) while
// the tile is staged, so the diagonal never exists as a matrix.  The chain
// product X <- E diag(d_l) X, the slice wrap G <- E diag(d) G diag(1/d) E^{-1}
// and the UDV update V <- diag(1/D) R (Pi^T V) are all instances.
//
// Tiling: a workgroup computes a TM x TN tile of C with GM x GN wavefronts;
// each wavefront owns WM x WN blocks of 16 x 16 accumulated by MFMA.  The
// K dimension is staged through LDS TK = 16 at a time, with the next stage
// prefetched into registers while the current one is consumed.
#include "slq_internal.h"

namespace slq {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int TK = 16;

// Position of accumulator element r of lane `lane` inside a 16 x 16 block of
// v_mfma_f64_16x16x4_f64 (operands: lane l holds A[l%16][l/16] and
// B[l/16][l%16]; result register r of lane l is D[l/16 + 4r][l%16]).
__device__ __forceinline__ int acc_row(int lane, int r) { return (lane >> 4) + 4 * r; }
__device__ __forceinline__ int acc_col(int lane, int r) { return lane & 15; }

template <int WM, int WN, int GM, int GN, bool TA, bool TB>
__global__ __launch_bounds__(64 * GM * GN) void k_gemm(GemmArgs g) {
  constexpr int TM = 16 * WM * GM, TN = 16 * WN * GN, NT = 64 * GM * GN;
  constexpr int APT = (TM * TK + NT - 1) / NT, BPT = (TK * TN + NT - 1) / NT;
  constexpr int PADM = TM + 1, PADN = TN + 1;
  __shared__ double As[TK][PADM];
  __shared__ double Bs[TK][PADN];

  const int b = blockIdx.z;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / GN) * WM * 16, wn0 = (wave % GN) * WN * 16;

  const double* A = g.A + (long)b * g.strideA;
  const double* B = g.B + (long)b * g.strideB;
  const int8_t* S = g.S ? g.S + (long)b * g.strideS + (long)g.slice * g.K : nullptr;
  double rpos = 0.0, rneg = 0.0;
  if (S) {
    rpos = g.consts[g.inv_scale ? 1 : 0];  // s = +1
    rneg = g.consts[g.inv_scale ? 0 : 1];  // s = -1
  }

  d4_t acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

  double ra[APT], rb[BPT];
  int kbeg = 0;
  if (g.a_upper) kbeg = (m0 / TK) * TK;

  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < APT; ++t) {
      const int idx = tid + t * NT;
      double v = 0.0;
      if (idx < TM * TK) {
        int mm, kk;
        if (TA) {
          mm = idx % TM;
          kk = idx / TM;
        } else {
          kk = idx % TK;
          mm = idx / TK;
        }
        const int gm = m0 + mm, gk = k0 + kk;
        if (gm < g.M && gk < g.K && !(g.a_upper && gk < gm))
          v = TA ? A[(long)gk * g.lda + gm] : A[(long)gm * g.lda + gk];
      }
      ra[t] = v;
    }
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
      const int idx = tid + t * NT;
      double v = 0.0;
      if (idx < TK * TN) {
        int nn, kk;
        if (TB) {
          kk = idx % TK;
          nn = idx / TK;
        } else {
          nn = idx % TN;
          kk = idx / TN;
        }
        const int gn = n0 + nn, gk = k0 + kk;
        if (gn < g.N && gk < g.K) {
          v = TB ? B[(long)gn * g.ldb + gk] : B[(long)gk * g.ldb + gn];
          if (S) v *= (S[gk] > 0) ? rpos : rneg;
        }
      }
      rb[t] = v;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int t = 0; t < APT; ++t) {
      const int idx = tid + t * NT;
      if (idx < TM * TK) {
        int mm, kk;
        if (TA) {
          mm = idx % TM;
          kk = idx / TM;
        } else {
          kk = idx % TK;
          mm = idx / TK;
        }
        As[kk][mm] = ra[t];
      }
    }
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
      const int idx = tid + t * NT;
      if (idx < TK * TN) {
        int nn, kk;
        if (TB) {
          kk = idx % TK;
          nn = idx / TK;
        } else {
          nn = idx % TN;
          kk = idx / TN;
        }
        Bs[kk][nn] = rb[t];
      }
    }
  };

  if (kbeg < g.K) load(kbeg);
  for (int k0 = kbeg; k0 < g.K; k0 += TK) {
    __syncthreads();
    store();
    __syncthreads();
    if (k0 + TK < g.K) load(k0 + TK);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      const int kr = ks + (lane >> 4);
      double af[WM], bf[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) af[i] = As[kr][wm0 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < WN; ++j) bf[j] = Bs[kr][wn0 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  }

  double* C = g.C + (long)b * g.strideC;
  const double* RS = g.rowscale ? g.rowscale + (long)b * g.strideRS : nullptr;
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm0 + i * 16 + acc_row(lane, r);
        const int gn = n0 + wn0 + j * 16 + acc_col(lane, r);
        if (gm < g.M && gn < g.N) {
          double v = g.alpha * acc[i][j][r];
          if (RS) v *= RS[gm];
          const long o = (long)gm * g.ldc + gn;
          C[o] = (g.beta != 0.0) ? v + g.beta * C[o] : v;
        }
      }
}

template <int WM, int WN, int GM, int GN>
static int run(const GemmArgs& a, bool ta, bool tb, hipStream_t st) {
  constexpr int TM = 16 * WM * GM, TN = 16 * WN * GN;
  dim3 grid((a.N + TN - 1) / TN, (a.M + TM - 1) / TM, a.batch);
  dim3 block(64 * GM * GN);
  if (!ta && !tb) k_gemm<WM, WN, GM, GN, false, false><<<grid, block, 0, st>>>(a);
  else if (ta && !tb) k_gemm<WM, WN, GM, GN, true, false><<<grid, block, 0, st>>>(a);
  else if (!ta && tb) k_gemm<WM, WN, GM, GN, false, true><<<grid, block, 0, st>>>(a);
  else k_gemm<WM, WN, GM, GN, true, true><<<grid, block, 0, st>>>(a);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

// Tile choice: the largest square tile that divides both M and N, else 64 x 64
// with ragged edges.
int launch_gemm(const GemmArgs& a, bool ta, bool tb, hipStream_t st) {
  if (a.batch <= 0 || a.M <= 0 || a.N <= 0) return SLQ_OK;
  auto divides = [&](int t) { return a.M % t == 0 && a.N % t == 0; };
  if (a.M >= 128 && divides(128)) return run<4, 4, 2, 2>(a, ta, tb, st);
  if (a.M >= 96 && divides(96)) return run<3, 3, 2, 2>(a, ta, tb, st);
  if (a.M >= 80 && divides(80)) return run<5, 1, 1, 5>(a, ta, tb, st);
  if (a.M >= 64 && divides(64)) return run<2, 2, 2, 2>(a, ta, tb, st);
  if (a.M >= 48 && divides(48)) return run<3, 1, 1, 3>(a, ta, tb, st);
  if (a.M <= 16 && a.N <= 16) return run<1, 1, 1, 1>(a, ta, tb, st);
  if (a.M <= 32 && a.N <= 32) return run<1, 1, 2, 2>(a, ta, tb, st);
  return run<2, 2, 2, 2>(a, ta, tb, st);
}

}  // namespace slq
