// Reduced-precision chain product: X <- E diag(d_l) X with FP32 or BF16
// operands and FP32 accumulation on the matrix cores, X kept in FP32 between
// slices.  The stabilisation (QR/UDV), the final LU and the log-det stay FP64;
// the chain block is widened to FP64 before each QR.
//
//   FP32: v_mfma_f32_16x16x4_f32  (lane l: A[l%16][l/16], B[l/16][l%16])
//   BF16: v_mfma_f32_16x16x32_bf16 (lane l: A[l%16][8(l/16)..+7], B[8(l/16)..+7][l%16])
//   result register r of lane l: D[4(l/16) + r][l%16] for both.
// Operands are rounded to the operand type (round to nearest even) when they
// are staged into LDS, i.e. at every GEMM of the chain.
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
