// Reduced-precision chain product: X <- E diag(d_l) X with FP32 or BF16
// operands and FP32 accumulation on the matrix cores, X kept in FP32 between
// slices.  The stabilisation (QR/UDV), the final LU and the log-det stay FP64;
// the chain block is widened to FP64 before each QR.
//
//   FP32: v_mfma_f32_16x16x4_f32  (lane l: A[l%16][l/16], B[l/16][l%16])
//   BF16: v_mfma_f32_16x16x32_bf16 (lane l: A[l%16][8(l/16)..+7], B[8(l/16)..+7][l%16])
//   result register r of lane l: D[4(l/16) + r][l%16] for both.
// Operands are rounded to the operand type (round to nearest even) when they
// are staged into LDS, i.e. at every GEMM of the chain.  For BF16 with N a
// multiple of 8 the chain instead stays in BF16 between slices, transposed
// and already scaled by the next slice's field (k_gemm_bf16t below): the same
// operand values, read with 16-byte loads.
#include <algorithm>

#include "slq_internal.h"

namespace slq {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

constexpr int LP_NXCD = 8;

template <typename T>
__device__ __forceinline__ float to_f(T v) {
  return (float)v;
}

// FP32 operands, TK = 16: LDS As[k][m], Bs[k][n] (as the FP64 kernel).
template <int WM, int WN, int GM, int GN, typename TB_T>
__global__ __launch_bounds__(64 * GM * GN) void k_gemm_f32(LpArgs g, int ntm, int ntn) {
  constexpr int TK = 16;
  constexpr int TM = 16 * WM * GM, TN = 16 * WN * GN, NT = 64 * GM * GN;
  constexpr int APT = (TM * TK + NT - 1) / NT, BPT = (TK * TN + NT - 1) / NT;
  __shared__ float As[2][TK][TM + 4];
  __shared__ float Bs[2][TK][TN + 4];
  const int tpi = ntm * ntn, gid = blockIdx.x, x = gid % LP_NXCD, j = gid / LP_NXCD;
  const int b = (j / tpi) * LP_NXCD + x;
  if (b >= g.batch) return;
  const int tile = j % tpi, tn = tile / ntm, tmi = tile % ntm;
  const int m0 = tmi * TM, n0 = tn * TN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / GN) * WM * 16, wn0 = (wave % GN) * WN * 16;
  const float* A = g.A;
  const TB_T* B = (const TB_T*)g.B + (long)b * g.strideB;
  const int8_t* S = g.S + (long)b * g.strideS + (long)g.slice * g.K;
  const float rpos = (float)g.consts[0], rneg = (float)g.consts[1];
  f4_t acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int jj = 0; jj < WN; ++jj) acc[i][jj] = f4_t{0.f, 0.f, 0.f, 0.f};
  float ra[APT], rb[BPT];
  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < APT; ++t) {
      const int idx = tid + t * NT;
      float v = 0.f;
      if (idx < TM * TK) {
        const int mm = idx / TK, kk = idx % TK, gm = m0 + mm, gk = k0 + kk;
        if (gm < g.M && gk < g.K) v = A[(long)gm * g.lda + gk];
      }
      ra[t] = v;
    }
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
      const int idx = tid + t * NT;
      float v = 0.f;
      if (idx < TK * TN) {
        const int nn = idx % TN, kk = idx / TN, gn = n0 + nn, gk = k0 + kk;
        if (gn < g.N && gk < g.K) v = to_f(B[(long)gk * g.ldb + gn]) * ((S[gk] > 0) ? rpos : rneg);
      }
      rb[t] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int t = 0; t < APT; ++t) {
      const int idx = tid + t * NT;
      if (idx < TM * TK) As[buf][idx % TK][idx / TK] = ra[t];
    }
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
      const int idx = tid + t * NT;
      if (idx < TK * TN) Bs[buf][idx / TN][idx % TN] = rb[t];
    }
  };
  load(0);
  store(0);
  __syncthreads();
  int cur = 0;
  for (int k0 = 0; k0 < g.K; k0 += TK) {
    const bool more = k0 + TK < g.K;
    if (more) load(k0 + TK);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      const int kr = ks + (lane >> 4);
      float af[WM], bf[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) af[i] = As[cur][kr][wm0 + i * 16 + (lane & 15)];
#pragma unroll
      for (int jj = 0; jj < WN; ++jj) bf[jj] = Bs[cur][kr][wn0 + jj * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int jj = 0; jj < WN; ++jj)
          acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[jj], acc[i][jj], 0, 0, 0);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  float* C = g.C + (long)b * g.strideC;
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int jj = 0; jj < WN; ++jj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm0 + i * 16 + 4 * (lane >> 4) + r, gn = n0 + wn0 + jj * 16 + (lane & 15);
        if (gm < g.M && gn < g.N) C[(long)gm * g.ldc + gn] = acc[i][jj][r];
      }
}

// BF16 operands, TK = 32: LDS As[m][k], Bs[n][k] (k contiguous: one 16-byte
// read gives a lane its eight consecutive k).
template <int WM, int WN, int GM, int GN, typename TB_T>
__global__ __launch_bounds__(64 * GM * GN) void k_gemm_bf16(LpArgs g, int ntm, int ntn) {
  constexpr int TK = 32, KP = TK + 8;
  constexpr int TM = 16 * WM * GM, TN = 16 * WN * GN, NT = 64 * GM * GN;
  constexpr int APT = (TM * TK + NT - 1) / NT, BPT = (TK * TN + NT - 1) / NT;
  __shared__ __attribute__((aligned(16))) __bf16 As[2][TM][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][TN][KP];
  const int tpi = ntm * ntn, gid = blockIdx.x, x = gid % LP_NXCD, j = gid / LP_NXCD;
  const int b = (j / tpi) * LP_NXCD + x;
  if (b >= g.batch) return;
  const int tile = j % tpi, tn = tile / ntm, tmi = tile % ntm;
  const int m0 = tmi * TM, n0 = tn * TN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / GN) * WM * 16, wn0 = (wave % GN) * WN * 16;
  const float* A = g.A;
  const TB_T* B = (const TB_T*)g.B + (long)b * g.strideB;
  const int8_t* S = g.S + (long)b * g.strideS + (long)g.slice * g.K;
  const float rpos = (float)g.consts[0], rneg = (float)g.consts[1];
  f4_t acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int jj = 0; jj < WN; ++jj) acc[i][jj] = f4_t{0.f, 0.f, 0.f, 0.f};
  float ra[APT], rb[BPT];
  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < APT; ++t) {
      const int idx = tid + t * NT;
      float v = 0.f;
      if (idx < TM * TK) {
        const int mm = idx / TK, kk = idx % TK, gm = m0 + mm, gk = k0 + kk;
        if (gm < g.M && gk < g.K) v = A[(long)gm * g.lda + gk];
      }
      ra[t] = v;
    }
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
      const int idx = tid + t * NT;
      float v = 0.f;
      if (idx < TK * TN) {
        const int nn = idx % TN, kk = idx / TN, gn = n0 + nn, gk = k0 + kk;
        if (gn < g.N && gk < g.K) v = to_f(B[(long)gk * g.ldb + gn]) * ((S[gk] > 0) ? rpos : rneg);
      }
      rb[t] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int t = 0; t < APT; ++t) {
      const int idx = tid + t * NT;
      if (idx < TM * TK) As[buf][idx / TK][idx % TK] = (__bf16)ra[t];
    }
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
      const int idx = tid + t * NT;
      if (idx < TK * TN) Bs[buf][idx % TN][idx / TN] = (__bf16)rb[t];
    }
  };
  load(0);
  store(0);
  __syncthreads();
  int cur = 0;
  const int kq = 8 * (lane >> 4);
  for (int k0 = 0; k0 < g.K; k0 += TK) {
    const bool more = k0 + TK < g.K;
    if (more) load(k0 + TK);
    bf8_t af[WM], bf[WN];
#pragma unroll
    for (int i = 0; i < WM; ++i) af[i] = *(const bf8_t*)&As[cur][wm0 + i * 16 + (lane & 15)][kq];
#pragma unroll
    for (int jj = 0; jj < WN; ++jj) bf[jj] = *(const bf8_t*)&Bs[cur][wn0 + jj * 16 + (lane & 15)][kq];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int jj = 0; jj < WN; ++jj)
        acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[jj], acc[i][jj], 0, 0, 0);
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  float* C = g.C + (long)b * g.strideC;
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int jj = 0; jj < WN; ++jj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm0 + i * 16 + 4 * (lane >> 4) + r, gn = n0 + wn0 + jj * 16 + (lane & 15);
        if (gm < g.M && gn < g.N) C[(long)gm * g.ldc + gn] = acc[i][jj][r];
      }
}

template <int WM, int WN, int GM, int GN>
static int run_lp(const LpArgs& a, int prec, bool b_is_f64, hipStream_t st) {
  constexpr int TM = 16 * WM * GM, TN = 16 * WN * GN;
  const int ntm = (a.M + TM - 1) / TM, ntn = (a.N + TN - 1) / TN;
  const long groups = ((long)a.batch + LP_NXCD - 1) / LP_NXCD * LP_NXCD * ntm * ntn;
  dim3 grid((unsigned)groups), block(64 * GM * GN);
  if (prec == SLQ_PREC_FP32) {
    if (b_is_f64) k_gemm_f32<WM, WN, GM, GN, double><<<grid, block, 0, st>>>(a, ntm, ntn);
    else k_gemm_f32<WM, WN, GM, GN, float><<<grid, block, 0, st>>>(a, ntm, ntn);
  } else {
    if (b_is_f64) k_gemm_bf16<WM, WN, GM, GN, double><<<grid, block, 0, st>>>(a, ntm, ntn);
    else k_gemm_bf16<WM, WN, GM, GN, float><<<grid, block, 0, st>>>(a, ntm, ntn);
  }
  SLQ_LAUNCHED();
  return SLQ_OK;
}

int launch_gemm_lp(const LpArgs& a, int prec, bool b_is_f64, hipStream_t st) {
  if (a.batch <= 0) return SLQ_OK;
  auto divides = [&](int t) { return a.M % t == 0 && a.N % t == 0; };
  if (a.M <= 16 && a.N <= 16) return run_lp<1, 1, 1, 1>(a, prec, b_is_f64, st);
  if (a.M >= 128 && divides(128)) return run_lp<4, 4, 2, 2>(a, prec, b_is_f64, st);
  if (a.M >= 96 && divides(96)) return run_lp<3, 3, 2, 2>(a, prec, b_is_f64, st);
  if (a.M >= 80 && divides(80)) return run_lp<5, 1, 1, 5>(a, prec, b_is_f64, st);
  if (a.M >= 64 && divides(64)) return run_lp<2, 2, 2, 2>(a, prec, b_is_f64, st);
  if (a.M >= 48 && divides(48)) return run_lp<3, 1, 1, 3>(a, prec, b_is_f64, st);
  return run_lp<2, 2, 2, 2>(a, prec, b_is_f64, st);
}

// X32[b] = E diag(d_slice) in FP32 (the first slice of a chain).
__global__ void k_first_slice_f32(int N, const double* __restrict__ E, const int8_t* __restrict__ s, long strideS,
                                  int slice, const double* __restrict__ consts, float* __restrict__ X) {
  const int b = blockIdx.y;
  const long NN = (long)N * N;
  const int8_t* sb = s + (long)b * strideS + (long)slice * N;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < NN; idx += (long)gridDim.x * blockDim.x) {
    const int j = (int)(idx % N);
    X[b * NN + idx] = (float)(E[idx] * (sb[j] > 0 ? consts[0] : consts[1]));
  }
}

__global__ void k_f32_to_f64(const float* __restrict__ a, double* __restrict__ b, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[i] = (double)a[i];
}

__global__ void k_f64_to_f32(const double* __restrict__ a, float* __restrict__ b, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

int launch_first_slice_f32(Plan& p, int batch, const int8_t* s, long strideS, int slice, float* X, hipStream_t st) {
  const long NN = (long)p.n * p.n;
  dim3 grid((unsigned)std::min<long>((NN + 255) / 256, 1024), batch);
  k_first_slice_f32<<<grid, 256, 0, st>>>(p.n, p.E, s, strideS, slice, p.consts, X);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

int launch_widen(const float* a, double* b, long n, hipStream_t st) {
  k_f32_to_f64<<<(unsigned)std::max<long>(1, std::min<long>((n + 255) / 256, 4096)), 256, 0, st>>>(a, b, n);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

int launch_narrow(const double* a, float* b, long n, hipStream_t st) {
  k_f64_to_f32<<<(unsigned)std::max<long>(1, std::min<long>((n + 255) / 256, 4096)), 256, 0, st>>>(a, b, n);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

}  // namespace slq

namespace slq {

// ---------------------------------------------------------------------------
// BF16 chain with k-contiguous operands.  Between the slices of a block the
// chain matrix is kept transposed in BF16 with the next slice's field factor
// already applied, Y^T[n][k] = bf16(d_next[k] X[k][n]): the B operand of the
// next product X' = E Y is then read like A = E (bf16, [m][k]), both with
// 16-byte loads, and the values are those the FP32-X path rounds to (the FP32
// accumulator times d, rounded once to BF16).  The last slice of a block
// writes X in FP64 for the QR.  Needs N % 8 == 0.

struct LpTArgs {
  int M, N, K;
  const __bf16* A;  // [M][K]
  long lda;
  const __bf16* BT;  // [batch] [N][K]
  long ldbt, strideBT;
  void* C;  // OUT 0: bf16 [batch] [N][M] (ldc = M), scaled rows; OUT 1: double [batch] [M][N]
  long ldc, strideC;
  const int8_t* S;  // fields [batch][L][M]; OUT 0 scales row m by d of slice `slice_next`
  long strideS;
  int slice_next;
  const double* consts;
  int batch;
};

typedef unsigned int u4_t __attribute__((ext_vector_type(4)));

template <int WM, int WN, int GM, int GN, int OUT>
__global__ __launch_bounds__(64 * GM * GN) void k_gemm_bf16t(LpTArgs g, int ntm, int ntn) {
  constexpr int TK = 32, KP = TK + 8;  // rows of 80 bytes: 16-byte aligned
  constexpr int TM = 16 * WM * GM, TN = 16 * WN * GN, NT = 64 * GM * GN;
  constexpr int AV = TM * TK / 8, BV = TN * TK / 8;  // 16-byte vectors per stage
  constexpr int APT = (AV + NT - 1) / NT, BPT = (BV + NT - 1) / NT;
  __shared__ __attribute__((aligned(16))) __bf16 As[2][TM][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][TN][KP];
  const int tpi = ntm * ntn, gid = blockIdx.x, x = gid % LP_NXCD, j = gid / LP_NXCD;
  const int b = (j / tpi) * LP_NXCD + x;
  if (b >= g.batch) return;
  const int tile = j % tpi, tn = tile / ntm, tmi = tile % ntm;
  const int m0 = tmi * TM, n0 = tn * TN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / GN) * WM * 16, wn0 = (wave % GN) * WN * 16;
  const __bf16* A = g.A;
  const __bf16* BT = g.BT + (long)b * g.strideBT;
  f4_t acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int jj = 0; jj < WN; ++jj) acc[i][jj] = f4_t{0.f, 0.f, 0.f, 0.f};
  u4_t ra[APT], rb[BPT];
  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < APT; ++t) {
      const int v = tid + t * NT;
      u4_t w = u4_t{0u, 0u, 0u, 0u};
      if (v < AV) {
        const int mm = v / (TK / 8), kq = v % (TK / 8), gm = m0 + mm, gk = k0 + 8 * kq;
        if (gm < g.M && gk < g.K) w = *(const u4_t*)(A + (long)gm * g.lda + gk);
      }
      ra[t] = w;
    }
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
      const int v = tid + t * NT;
      u4_t w = u4_t{0u, 0u, 0u, 0u};
      if (v < BV) {
        const int nn = v / (TK / 8), kq = v % (TK / 8), gn = n0 + nn, gk = k0 + 8 * kq;
        if (gn < g.N && gk < g.K) w = *(const u4_t*)(BT + (long)gn * g.ldbt + gk);
      }
      rb[t] = w;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int t = 0; t < APT; ++t) {
      const int v = tid + t * NT;
      if (v < AV) *(u4_t*)&As[buf][v / (TK / 8)][8 * (v % (TK / 8))] = ra[t];
    }
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
      const int v = tid + t * NT;
      if (v < BV) *(u4_t*)&Bs[buf][v / (TK / 8)][8 * (v % (TK / 8))] = rb[t];
    }
  };
  load(0);
  store(0);
  __syncthreads();
  int cur = 0;
  const int kq = 8 * (lane >> 4);
  for (int k0 = 0; k0 < g.K; k0 += TK) {
    const bool more = k0 + TK < g.K;
    if (more) load(k0 + TK);
    bf8_t af[WM], bf[WN];
#pragma unroll
    for (int i = 0; i < WM; ++i) af[i] = *(const bf8_t*)&As[cur][wm0 + i * 16 + (lane & 15)][kq];
#pragma unroll
    for (int jj = 0; jj < WN; ++jj) bf[jj] = *(const bf8_t*)&Bs[cur][wn0 + jj * 16 + (lane & 15)][kq];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int jj = 0; jj < WN; ++jj)
        acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[jj], acc[i][jj], 0, 0, 0);
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  if constexpr (OUT == 1) {
    double* C = (double*)g.C + (long)b * g.strideC;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int jj = 0; jj < WN; ++jj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gm = m0 + wm0 + i * 16 + 4 * (lane >> 4) + r, gn = n0 + wn0 + jj * 16 + (lane & 15);
          if (gm < g.M && gn < g.N) C[(long)gm * g.ldc + gn] = (double)acc[i][jj][r];
        }
  } else {
    __bf16* C = (__bf16*)g.C + (long)b * g.strideC;
    const int8_t* S = g.S + (long)b * g.strideS + (long)g.slice_next * g.M;
    const float rpos = (float)g.consts[0], rneg = (float)g.consts[1];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int jj = 0; jj < WN; ++jj) {
        const int gm = m0 + wm0 + i * 16 + 4 * (lane >> 4), gn = n0 + wn0 + jj * 16 + (lane & 15);
        if (gm < g.M && gn < g.N) {  // M % 4 == 0: the four rows gm..gm+3 are all inside
          typedef __bf16 bf4_t __attribute__((ext_vector_type(4)));
          bf4_t o;
#pragma unroll
          for (int r = 0; r < 4; ++r) o[r] = (__bf16)(acc[i][jj][r] * ((S[gm + r] > 0) ? rpos : rneg));
          *(bf4_t*)(C + (long)gn * g.ldc + gm) = o;
        }
      }
  }
}

template <int WM, int WN, int GM, int GN>
static void run_bf16t(const LpTArgs& a, int out, hipStream_t st) {
  constexpr int TM = 16 * WM * GM, TN = 16 * WN * GN;
  const int ntm = (a.M + TM - 1) / TM, ntn = (a.N + TN - 1) / TN;
  const long groups = ((long)a.batch + LP_NXCD - 1) / LP_NXCD * LP_NXCD * ntm * ntn;
  dim3 grid((unsigned)groups), block(64 * GM * GN);
  if (out == 1)
    k_gemm_bf16t<WM, WN, GM, GN, 1><<<grid, block, 0, st>>>(a, ntm, ntn);
  else
    k_gemm_bf16t<WM, WN, GM, GN, 0><<<grid, block, 0, st>>>(a, ntm, ntn);
}

int launch_gemm_bf16t(const LpTArgs& a, int out, hipStream_t st) {
  if (a.batch <= 0) return SLQ_OK;
  if (a.M % 8 != 0 || a.K % 8 != 0 || a.lda % 8 != 0 || a.ldbt % 8 != 0) {
    set_error("the BF16 chain with k-contiguous operands needs multiples of 8");
    return SLQ_ERR_ARG;
  }
  if (a.M % 160 == 0 && a.N % 160 == 0)
    run_bf16t<5, 5, 2, 2>(a, out, st);
  else if (a.M <= 64 && a.N <= 64)
    run_bf16t<2, 2, 2, 2>(a, out, st);
  else
    run_bf16t<4, 4, 2, 2>(a, out, st);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

// BT[b][n][k] = T(d[k] X[b][k][n]) (X FP64 row-major, the product formed in
// FP32), or T(d[k]) on the diagonal when X is null (the identity); 32 x 32
// tiles through LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_bt_prepare(int N, const double* __restrict__ X, long strideX,
                                                    const int8_t* __restrict__ S, long strideS, int slice,
                                                    const double* __restrict__ consts, T* __restrict__ BT) {
  __shared__ float t[32][33];
  const int b = blockIdx.z, k0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int8_t* sb = S + (long)b * strideS + (long)slice * N;
  const float rpos = (float)consts[0], rneg = (float)consts[1];
  for (int r = ty; r < 32; r += 8) {  // rows k, columns n
    const int k = k0 + r, n = n0 + tx;
    float v = 0.f;
    if (k < N && n < N) {
      const double x = X ? X[(long)b * strideX + (long)k * N + n] : (k == n ? 1.0 : 0.0);
      v = (float)x * ((sb[k] > 0) ? rpos : rneg);
    }
    t[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {  // rows n, columns k
    const int n = n0 + r, k = k0 + tx;
    if (n < N && k < N) BT[(long)b * N * N + (long)n * N + k] = (T)t[tx][r];
  }
}

int launch_bt_prepare(int N, int batch, const double* X, long strideX, const int8_t* S, long strideS, int slice,
                      const double* consts, void* BT, int prec, hipStream_t st) {
  dim3 grid((unsigned)((N + 31) / 32), (unsigned)((N + 31) / 32), (unsigned)batch);
  if (prec == SLQ_PREC_BF16)
    k_bt_prepare<__bf16><<<grid, 256, 0, st>>>(N, X, strideX, S, strideS, slice, consts, (__bf16*)BT);
  else
    k_bt_prepare<float><<<grid, 256, 0, st>>>(N, X, strideX, S, strideS, slice, consts, (float*)BT);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

// The FP32 chain with k-contiguous operands: the same scheme with FP32 storage
// (Y^T = (d_next X)^T in FP32, E32), v_mfma_f32_16x16x4_f32, 16-byte loads of
// four k; LDS rows of 20 floats keep the 16 rows a wave reads on distinct banks.
template <int WM, int WN, int GM, int GN, int OUT>
__global__ __launch_bounds__(64 * GM * GN) void k_gemm_f32t(LpTArgs g, const float* __restrict__ A,
                                                            const float* __restrict__ BTall, int ntm, int ntn) {
  constexpr int TK = 16, KP = TK + 4;
  constexpr int TM = 16 * WM * GM, TN = 16 * WN * GN, NT = 64 * GM * GN;
  constexpr int AV = TM * TK / 4, BV = TN * TK / 4;  // 16-byte vectors per stage
  constexpr int APT = (AV + NT - 1) / NT, BPT = (BV + NT - 1) / NT;
  __shared__ __attribute__((aligned(16))) float As[2][TM][KP];
  __shared__ __attribute__((aligned(16))) float Bs[2][TN][KP];
  const int tpi = ntm * ntn, gid = blockIdx.x, x = gid % LP_NXCD, j = gid / LP_NXCD;
  const int b = (j / tpi) * LP_NXCD + x;
  if (b >= g.batch) return;
  const int tile = j % tpi, tn = tile / ntm, tmi = tile % ntm;
  const int m0 = tmi * TM, n0 = tn * TN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / GN) * WM * 16, wn0 = (wave % GN) * WN * 16;
  const float* BT = BTall + (long)b * g.strideBT;
  f4_t acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int jj = 0; jj < WN; ++jj) acc[i][jj] = f4_t{0.f, 0.f, 0.f, 0.f};
  f4_t ra[APT], rb[BPT];
  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < APT; ++t) {
      const int v = tid + t * NT;
      f4_t w = f4_t{0.f, 0.f, 0.f, 0.f};
      if (v < AV) {
        const int mm = v / (TK / 4), kq = v % (TK / 4), gm = m0 + mm, gk = k0 + 4 * kq;
        if (gm < g.M && gk < g.K) w = *(const f4_t*)(A + (long)gm * g.lda + gk);
      }
      ra[t] = w;
    }
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
      const int v = tid + t * NT;
      f4_t w = f4_t{0.f, 0.f, 0.f, 0.f};
      if (v < BV) {
        const int nn = v / (TK / 4), kq = v % (TK / 4), gn = n0 + nn, gk = k0 + 4 * kq;
        if (gn < g.N && gk < g.K) w = *(const f4_t*)(BT + (long)gn * g.ldbt + gk);
      }
      rb[t] = w;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int t = 0; t < APT; ++t) {
      const int v = tid + t * NT;
      if (v < AV) *(f4_t*)&As[buf][v / (TK / 4)][4 * (v % (TK / 4))] = ra[t];
    }
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
      const int v = tid + t * NT;
      if (v < BV) *(f4_t*)&Bs[buf][v / (TK / 4)][4 * (v % (TK / 4))] = rb[t];
    }
  };
  load(0);
  store(0);
  __syncthreads();
  int cur = 0;
  for (int k0 = 0; k0 < g.K; k0 += TK) {
    const bool more = k0 + TK < g.K;
    if (more) load(k0 + TK);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      const int kr = ks + (lane >> 4);
      float af[WM], bf[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) af[i] = As[cur][wm0 + i * 16 + (lane & 15)][kr];
#pragma unroll
      for (int jj = 0; jj < WN; ++jj) bf[jj] = Bs[cur][wn0 + jj * 16 + (lane & 15)][kr];
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int jj = 0; jj < WN; ++jj)
          acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[jj], acc[i][jj], 0, 0, 0);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  if constexpr (OUT == 1) {
    double* C = (double*)g.C + (long)b * g.strideC;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int jj = 0; jj < WN; ++jj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gm = m0 + wm0 + i * 16 + 4 * (lane >> 4) + r, gn = n0 + wn0 + jj * 16 + (lane & 15);
          if (gm < g.M && gn < g.N) C[(long)gm * g.ldc + gn] = (double)acc[i][jj][r];
        }
  } else {
    float* C = (float*)g.C + (long)b * g.strideC;
    const int8_t* S = g.S + (long)b * g.strideS + (long)g.slice_next * g.M;
    const float rpos = (float)g.consts[0], rneg = (float)g.consts[1];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int jj = 0; jj < WN; ++jj) {
        const int gm = m0 + wm0 + i * 16 + 4 * (lane >> 4), gn = n0 + wn0 + jj * 16 + (lane & 15);
        if (gm < g.M && gn < g.N) {  // M % 4 == 0: the four rows gm..gm+3 are all inside
          f4_t o;
#pragma unroll
          for (int r = 0; r < 4; ++r) o[r] = acc[i][jj][r] * ((S[gm + r] > 0) ? rpos : rneg);
          *(f4_t*)(C + (long)gn * g.ldc + gm) = o;
        }
      }
  }
}

template <int WM, int WN, int GM, int GN>
static void run_f32t(const LpTArgs& a, const float* A, const float* BT, int out, hipStream_t st) {
  constexpr int TM = 16 * WM * GM, TN = 16 * WN * GN;
  const int ntm = (a.M + TM - 1) / TM, ntn = (a.N + TN - 1) / TN;
  const long groups = ((long)a.batch + LP_NXCD - 1) / LP_NXCD * LP_NXCD * ntm * ntn;
  dim3 grid((unsigned)groups), block(64 * GM * GN);
  if (out == 1)
    k_gemm_f32t<WM, WN, GM, GN, 1><<<grid, block, 0, st>>>(a, A, BT, ntm, ntn);
  else
    k_gemm_f32t<WM, WN, GM, GN, 0><<<grid, block, 0, st>>>(a, A, BT, ntm, ntn);
}

int launch_f32t_product(Plan& p, int batch, const void* BT, void* out, int out_f64, const int8_t* s, long strideS,
                        int slice_next, hipStream_t st) {
  const int N = p.n;
  const long NN = (long)N * N;
  if (N % 8 != 0) {
    set_error("the FP32 chain with k-contiguous operands needs N % 8 == 0");
    return SLQ_ERR_ARG;
  }
  LpTArgs a{};
  a.M = N;
  a.N = N;
  a.K = N;
  a.lda = N;
  a.ldbt = N;
  a.strideBT = NN;
  a.C = out;
  a.ldc = N;
  a.strideC = NN;
  a.S = s;
  a.strideS = strideS;
  a.slice_next = slice_next;
  a.consts = p.consts;
  a.batch = batch;
  if (batch <= 0) return SLQ_OK;
  if (N % 160 == 0)
    run_f32t<5, 5, 2, 2>(a, p.E32, (const float*)BT, out_f64, st);
  else if (N <= 64)
    run_f32t<2, 2, 2, 2>(a, p.E32, (const float*)BT, out_f64, st);
  else
    run_f32t<4, 4, 2, 2>(a, p.E32, (const float*)BT, out_f64, st);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

int launch_bf16t_product(Plan& p, int batch, const void* BT, void* out, int out_f64, const int8_t* s, long strideS,
                         int slice_next, hipStream_t st) {
  const int N = p.n;
  const long NN = (long)N * N;
  LpTArgs a{};
  a.M = N;
  a.N = N;
  a.K = N;
  a.A = (const __bf16*)p.E16;
  a.lda = N;
  a.BT = (const __bf16*)BT;
  a.ldbt = N;
  a.strideBT = NN;
  a.C = out;
  a.ldc = N;
  a.strideC = NN;
  a.S = s;
  a.strideS = strideS;
  a.slice_next = slice_next;
  a.consts = p.consts;
  a.batch = batch;
  return launch_gemm_bf16t(a, out_f64, st);
}

__global__ void k_f32_to_bf16(const float* __restrict__ a, __bf16* __restrict__ b, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[i] = (__bf16)a[i];
}

int launch_to_bf16(const float* a, void* b, long n, hipStream_t st) {
  k_f32_to_bf16<<<(unsigned)std::max<long>(1, std::min<long>((n + 255) / 256, 4096)), 256, 0, st>>>(
      a, (__bf16*)b, n);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

}  // namespace slq
