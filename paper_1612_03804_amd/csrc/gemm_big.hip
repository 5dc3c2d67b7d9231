// Batched FP64 GEMM for large tile-aligned products on the CDNA4 matrix cores
// (v_mfma_f64_16x16x4_f64); the general kernel, its tiles and the dispatch
// are in gemm.hip.  Built with the accumulators in VGPRs (the AGPR form
// copied all 64 accumulators of a lane between the register files at every
// K stage).
#include <cstdint>

#include "slq_internal.h"

namespace slq {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int NXCD = 8;

// position of accumulator element r of lane `lane` in a 16 x 16 block of
// v_mfma_f64_16x16x4_f64 (result register r of lane l is D[l/16 + 4r][l%16])
__device__ __forceinline__ int acc_row(int lane, int r) { return (lane >> 4) + 4 * r; }
__device__ __forceinline__ int acc_col(int lane, int r) { return lane & 15; }

// Large tile-aligned products (M and N multiples of 128, K of 16, even
// leading dimensions and 16-byte aligned operands: the trailing, Q-formation
// and V updates of the QR at N = 2304).  128 x 128 tiles of four wavefronts,
// each owning 64 x 64 of C (16 blocks, 64 accumulators per lane: 16 MFMAs per
// 8 LDS reads, two wavefronts per SIMD are enough); K staged 16 deep through
// two LDS buffers, the next stage's 16-byte global loads in flight while the
// current one is multiplied; no bounds checks.  MODE 1: upper-triangular A
// (K from the last tile down to the tile's diagonal, entries below it read as
// zero) with an optional row gather of B.
constexpr int BG_T = 128, BG_K = 16, BG_THREADS = 256, BG_PAD = BG_T + 2;

template <bool TA, int MODE>
__global__ __launch_bounds__(BG_THREADS) void k_gemm_big(GemmArgs g, int ntm, int ntn) {
  constexpr bool AUP = MODE == 1;
  __shared__ __attribute__((aligned(16))) double As[2][BG_K][BG_PAD];  // 16-byte stores of pairs
  __shared__ __attribute__((aligned(16))) double Bs[2][BG_K][BG_PAD];
  extern __shared__ int brow_s[];  // row gather of B: [K]
  const int tpi = ntm * ntn;
  const int gid = blockIdx.x;
  const int x = gid % NXCD, j = gid / NXCD;
  const int b = (j / tpi) * NXCD + x;
  if (b >= g.batch) return;
  const int tile = j % tpi;
  const int tn = tile / ntm, tmi = tile % ntm;
  const int m0 = tmi * BG_T, n0 = tn * BG_T;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * 64, wn0 = (wave & 1) * 64;
  const double* A = g.A + (long)b * g.strideA;
  const double* B = g.B + (long)b * g.strideB;
  const bool gather = AUP && g.brow;
  if (gather) {
    const int32_t* br = g.brow + (long)b * g.strideBrow;
    for (int k = tid; k < g.K; k += BG_THREADS) brow_s[k] = br[k];
    __syncthreads();
  }
  d4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) acc[i][jj] = d4_t{0.0, 0.0, 0.0, 0.0};
  // a stage: A 128 x 16 and B 16 x 128 as 1024 pairs of doubles each, 4 per thread
  double ra[8], rb[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int e = tid + p * BG_THREADS;
      double2 v;
      if constexpr (TA) {  // A stored [k][m]: pairs along m
        const int kr = e >> 6, mp = (e & 63) * 2;
        v = *(const double2*)(A + (long)(k0 + kr) * g.lda + m0 + mp);
      } else {  // A stored [m][k]: pairs along k
        const int row = e >> 3, kp = (e & 7) * 2;
        v = *(const double2*)(A + (long)(m0 + row) * g.lda + k0 + kp);
        if constexpr (AUP) {
          if (k0 + kp < m0 + row) v.x = 0.0;
          if (k0 + kp + 1 < m0 + row) v.y = 0.0;
        }
      }
      ra[2 * p] = v.x;
      ra[2 * p + 1] = v.y;
      const int kr = e >> 6, np = (e & 63) * 2;
      const int brw = gather ? brow_s[k0 + kr] : k0 + kr;
      const double2 w = *(const double2*)(B + (long)brw * g.ldb + n0 + np);
      rb[2 * p] = w.x;
      rb[2 * p + 1] = w.y;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int e = tid + p * BG_THREADS;
      if constexpr (TA) {
        const int kr = e >> 6, mp = (e & 63) * 2;
        *(double2*)&As[buf][kr][mp] = make_double2(ra[2 * p], ra[2 * p + 1]);
      } else {
        const int row = e >> 3, kp = (e & 7) * 2;
        As[buf][kp][row] = ra[2 * p];
        As[buf][kp + 1][row] = ra[2 * p + 1];
      }
      const int kr = e >> 6, np = (e & 63) * 2;
      *(double2*)&Bs[buf][kr][np] = make_double2(rb[2 * p], rb[2 * p + 1]);
    }
  };
  const int kbeg = AUP ? m0 : 0, klast = g.K - BG_K;
  const int kfirst = AUP ? klast : 0, kstep = AUP ? -BG_K : BG_K;
  const int nst = (g.K - kbeg) / BG_K;
  if (nst > 0) {
    load(kfirst);
    store(0);
  }
  __syncthreads();
  int cur = 0;
  for (int st = 0, k0 = kfirst; st < nst; ++st, k0 += kstep) {
    const bool more = st + 1 < nst;
    if (more) load(k0 + kstep);
#pragma unroll
    for (int ks = 0; ks < BG_K; ks += 4) {
      const int kr = ks + (lane >> 4);
      double af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = As[cur][kr][wm0 + i * 16 + (lane & 15)];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) bf[jj] = Bs[cur][kr][wn0 + jj * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          acc[i][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[jj], acc[i][jj], 0, 0, 0);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  double* C = g.C + (long)b * g.strideC;
  const double* RS = g.rowscale ? g.rowscale + (long)b * g.strideRS : nullptr;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gm = m0 + wm0 + i * 16 + acc_row(lane, r);
      const double rs = RS ? RS[gm] : 1.0;
      const bool zrow = gm < g.c_zero_rows;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int gn = n0 + wn0 + jj * 16 + acc_col(lane, r);
        double v = g.alpha * acc[i][jj][r] * rs;
        const long o = (long)gm * g.ldc + gn;
        if (g.beta != 0.0) {
          const double cin = g.c_ident ? (gm == gn ? 1.0 : 0.0) : (zrow ? 0.0 : C[o]);
          v += g.beta * cin;
        }
        C[o] = v;
      }
    }
}

// The 128 x 64 tiles of the general kernel (eight wavefronts of 32 x 32, K 8
// deep) without its bounds checks, loading pairs of doubles: for the rank-k
// updates of large blocks, where eight wavefronts per SIMD hide the short K.
constexpr int LN_M = 128, LN_N = 64, LN_K = 8, LN_THREADS = 512;

__global__ __launch_bounds__(LN_THREADS) void k_gemm_lean(GemmArgs g, int ntm, int ntn) {
  __shared__ __attribute__((aligned(16))) double As[2][LN_K][LN_M + 2];
  __shared__ __attribute__((aligned(16))) double Bs[2][LN_K][LN_N + 2];
  const int tpi = ntm * ntn;
  const int gid = blockIdx.x;
  const int x = gid % NXCD, j = gid / NXCD;
  const int b = (j / tpi) * NXCD + x;
  if (b >= g.batch) return;
  const int tile = j % tpi;
  const int tn = tile / ntm, tmi = tile % ntm;
  const int m0 = tmi * LN_M, n0 = tn * LN_N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * 32, wn0 = (wave & 1) * 32;
  const double* A = g.A + (long)b * g.strideA;
  const double* B = g.B + (long)b * g.strideB;
  d4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) acc[i][jj] = d4_t{0.0, 0.0, 0.0, 0.0};
  // a stage: A 128 x 8 as 512 pairs along k (one per thread), B 8 x 64 as 256 pairs along n
  const int arow = tid >> 2, akp = (tid & 3) * 2, bkr = (tid & 255) >> 5, bnp = (tid & 31) * 2;
  const bool bthr = tid < 256;
  double a0, a1, b0 = 0.0, b1 = 0.0;
  auto load = [&](int k0) {
    const double2 v = *(const double2*)(A + (long)(m0 + arow) * g.lda + k0 + akp);
    a0 = v.x;
    a1 = v.y;
    if (bthr) {
      const double2 w = *(const double2*)(B + (long)(k0 + bkr) * g.ldb + n0 + bnp);
      b0 = w.x;
      b1 = w.y;
    }
  };
  auto store = [&](int buf) {
    As[buf][akp][arow] = a0;
    As[buf][akp + 1][arow] = a1;
    if (bthr) *(double2*)&Bs[buf][bkr][bnp] = make_double2(b0, b1);
  };
  const int nst = g.K / LN_K;
  if (nst > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  int cur = 0;
  for (int st = 0; st < nst; ++st) {
    const bool more = st + 1 < nst;
    if (more) load((st + 1) * LN_K);
#pragma unroll
    for (int ks = 0; ks < LN_K; ks += 4) {
      const int kr = ks + (lane >> 4);
      double af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = As[cur][kr][wm0 + i * 16 + (lane & 15)];
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) bf[jj] = Bs[cur][kr][wn0 + jj * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
          acc[i][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[jj], acc[i][jj], 0, 0, 0);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  double* C = g.C + (long)b * g.strideC;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gm = m0 + wm0 + i * 16 + acc_row(lane, r);
      const bool zrow = gm < g.c_zero_rows;
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int gn = n0 + wn0 + jj * 16 + acc_col(lane, r);
        double v = g.alpha * acc[i][jj][r];
        const long o = (long)gm * g.ldc + gn;
        if (g.beta != 0.0) {
          const double cin = g.c_ident ? (gm == gn ? 1.0 : 0.0) : (zrow ? 0.0 : C[o]);
          v += g.beta * cin;
        }
        C[o] = v;
      }
    }
}

bool gemm_lean_ok(const GemmArgs& a, bool ta, bool tb) {
  auto al = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  if (ta || tb || a.S || a.a_upper || a.brow || a.rowscale) return false;
  if (a.M % LN_M || a.N % LN_N || a.K % LN_K || a.M <= 0 || a.N <= 0 || a.K <= 0) return false;
  return a.lda % 2 == 0 && a.ldb % 2 == 0 && a.strideA % 2 == 0 && a.strideB % 2 == 0 && al(a.A) && al(a.B);
}

int launch_gemm_lean(const GemmArgs& a, hipStream_t st) {
  const int ntm = a.M / LN_M, ntn = a.N / LN_N;
  const long groups = ((long)a.batch + NXCD - 1) / NXCD * NXCD * ntm * ntn;
  k_gemm_lean<<<dim3((unsigned)groups), LN_THREADS, 0, st>>>(a, ntm, ntn);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

bool gemm_big_ok(const GemmArgs& a, bool ta, bool tb) {
  auto al = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  if (tb || a.S || (a.a_upper && ta) || (a.brow && !a.a_upper)) return false;
  if (a.M % BG_T || a.N % BG_T || a.K % BG_K || a.M <= 0 || a.N <= 0 || a.K <= 0) return false;
  if (a.a_upper && a.M != a.K) return false;
  return a.lda % 2 == 0 && a.ldb % 2 == 0 && a.strideA % 2 == 0 && a.strideB % 2 == 0 && al(a.A) && al(a.B);
}

int launch_gemm_big(const GemmArgs& a, bool ta, hipStream_t st) {
  const int ntm = a.M / BG_T, ntn = a.N / BG_T;
  const long groups = ((long)a.batch + NXCD - 1) / NXCD * NXCD * ntm * ntn;
  const size_t lds = a.brow ? sizeof(int) * (size_t)a.K : 0;
  if (a.a_upper) {
    allow_max_lds((const void*)k_gemm_big<false, 1>);
    k_gemm_big<false, 1><<<dim3((unsigned)groups), BG_THREADS, lds, st>>>(a, ntm, ntn);
  } else if (ta) {
    k_gemm_big<true, 0><<<dim3((unsigned)groups), BG_THREADS, 0, st>>>(a, ntm, ntn);
  } else {
    k_gemm_big<false, 0><<<dim3((unsigned)groups), BG_THREADS, 0, st>>>(a, ntm, ntn);
  }
  SLQ_LAUNCHED();
  return SLQ_OK;
}

}  // namespace slq
