// Batched FP64 GEMM on the CDNA4 matrix cores (v_mfma_f64_16x16x4_f64).
//
//   C[b] = alpha * diag(rowscale_b) * op(A[b]) * diag(r_b) * op(B[b]) + beta * C[b]
//
// r_b is the field factor of one slice, exp(-+dtau xi s_{k,l}) ("Basics of
// DQMC": B_l = exp(-dtau K) exp(V(s_l))), applied to the rows of op(B) while
// the tile is staged, so the diagonal never exists as a matrix.  The chain
// product X <- E diag(d_l) X, the slice wrap G <- E diag(d) G diag(1/d) E^{-1},
// the UDV update V <- diag(1/D) R (Pi^T V) and the blocked-QR updates are all
// instances.
//
// Tiling: a workgroup computes a TM x TN tile of C with GM x GN wavefronts;
// each wavefront owns WM x WN blocks of 16 x 16 accumulated by MFMA.  K is
// staged through two LDS buffers TK deep: while the matrix cores work on one,
// the next tile is already in flight from memory into registers and is
// written to the other buffer, so there is one barrier per TK step.
// Workgroup order: the eight XCDs of the chip each own whole fields (a
// field's tiles are dispatched to one XCD, column panel by column panel), so
// the operand panels of a field are fetched into one L2 only.
#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "slq_internal.h"

namespace slq {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int NXCD = 8;

// Position of accumulator element r of lane `lane` inside a 16 x 16 block of
// v_mfma_f64_16x16x4_f64 (operands: lane l holds A[l%16][l/16] and
// B[l/16][l%16]; result register r of lane l is D[l/16 + 4r][l%16]).
__device__ __forceinline__ int acc_row(int lane, int r) { return (lane >> 4) + 4 * r; }
__device__ __forceinline__ int acc_col(int lane, int r) { return lane & 15; }

// MODE: 0 plain, 1 upper-triangular A (entries with k < m read as zero, the
// zero K tiles are skipped), 2 field-scaled rows of op(B) (the chain product
// and the wrap; a separate symbol so that profiles separate it).
template <int WM, int WN, int GM, int GN, int TK, bool TA, bool TB, int MODE>
__global__ __launch_bounds__(64 * GM * GN) void k_gemm(GemmArgs g, int ntm, int ntn) {
  constexpr bool AUP = MODE == 1, FS = MODE == 2, FSO = MODE == 3;
  constexpr int TM = 16 * WM * GM, TN = 16 * WN * GN, NT = 64 * GM * GN;
  constexpr int APT = (TM * TK + NT - 1) / NT, BPT = (TK * TN + NT - 1) / NT;
  constexpr int PADM = TM + 2, PADN = TN + 2;
  __shared__ double As[2][TK][PADM];
  __shared__ double Bs[2][TK][PADN];
  extern __shared__ int brow_s[];  // triangular mode with a row gather of B: [K]

  // XCD-aware decode of the linear workgroup id: item = field, tile in item
  const int tpi = ntm * ntn;
  const int gid = blockIdx.x;
  const int x = gid % NXCD, j = gid / NXCD;
  const int b = (j / tpi) * NXCD + x;
  if (b >= g.batch) return;
  const int tile = j % tpi;
  const int tn = tile / ntm, tmi = tile % ntm;  // column panel outer: its row tiles run back to back
  const int m0 = tmi * TM, n0 = tn * TN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / GN) * WM * 16, wn0 = (wave % GN) * WN * 16;

  const double* A = g.A + (long)b * g.strideA;
  const double* B = g.B + (long)b * g.strideB;
  const int8_t* S = (FS || FSO) ? g.S + (long)b * g.strideS + (long)g.slice * g.K : nullptr;
  double rpos = 0.0, rneg = 0.0;
  if (FS || FSO) {
    rpos = g.consts[g.inv_scale ? 1 : 0];  // s = +1
    rneg = g.consts[g.inv_scale ? 0 : 1];  // s = -1
  }

  d4_t acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int jj = 0; jj < WN; ++jj) acc[i][jj] = d4_t{0.0, 0.0, 0.0, 0.0};

  double ra[APT], rb[BPT];
  const int kbeg = AUP ? (m0 / TK) * TK : 0;
  const bool gather = AUP && g.brow;
  if (gather) {
    const int32_t* br = g.brow + (long)b * g.strideBrow;
    for (int k = tid; k < g.K; k += NT) brow_s[k] = br[k];
    __syncthreads();
  }

  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < APT; ++t) {
      const int idx = tid + t * NT;
      double v = 0.0;
      if (idx < TM * TK) {
        const int mm = TA ? idx % TM : idx / TK;
        const int kk = TA ? idx / TM : idx % TK;
        const int gm = m0 + mm, gk = k0 + kk;
        if (gm < g.M && gk < g.K && !(AUP && gk < gm))
          v = TA ? A[(long)gk * g.lda + gm] : A[(long)gm * g.lda + gk];
      }
      ra[t] = v;
    }
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
      const int idx = tid + t * NT;
      double v = 0.0;
      if (idx < TK * TN) {
        const int nn = TB ? idx / TK : idx % TN;
        const int kk = TB ? idx % TK : idx / TN;
        const int gn = n0 + nn, gk = k0 + kk;
        if (gn < g.N && gk < g.K) {
          v = TB ? B[(long)gn * g.ldb + gk] : B[(long)(gather ? brow_s[gk] : gk) * g.ldb + gn];
          if (FS) v *= (S[gk] > 0) ? rpos : rneg;
        }
      }
      rb[t] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int t = 0; t < APT; ++t) {
      const int idx = tid + t * NT;
      if (idx < TM * TK) {
        const int mm = TA ? idx % TM : idx / TK;
        const int kk = TA ? idx / TM : idx % TK;
        As[buf][kk][mm] = ra[t];
      }
    }
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
      const int idx = tid + t * NT;
      if (idx < TK * TN) {
        const int nn = TB ? idx / TK : idx % TN;
        const int kk = TB ? idx % TK : idx / TN;
        Bs[buf][kk][nn] = rb[t];
      }
    }
  };

  // A triangular A runs K backwards, from the last K tile down to the tile's
  // diagonal: every tile then starts at the same K, and the tiles resident
  // together read the same rows of op(B) at about the same time (forwards,
  // each row of tiles would start at its own diagonal and the B panels would
  // be fetched once per row of tiles).
  const int klast = g.K > 0 ? ((g.K - 1) / TK) * TK : 0;
  const int kfirst = AUP ? klast : kbeg, kstep = AUP ? -TK : TK;
  if (kbeg < g.K) {
    load(kfirst);
    store(0);
  }
  __syncthreads();
  int cur = 0;
  for (int k0 = kfirst; kbeg < g.K && (AUP ? k0 >= kbeg : k0 < g.K); k0 += kstep) {
    const bool more = AUP ? k0 - TK >= kbeg : k0 + TK < g.K;
    if (more) load(k0 + kstep);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      const int kr = ks + (lane >> 4);
      double af[WM], bf[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) af[i] = As[cur][kr][wm0 + i * 16 + (lane & 15)];
#pragma unroll
      for (int jj = 0; jj < WN; ++jj) bf[jj] = Bs[cur][kr][wn0 + jj * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int jj = 0; jj < WN; ++jj)
          acc[i][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[jj], acc[i][jj], 0, 0, 0);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }

  double* C = g.C + (long)b * g.strideC;
  const double* RS = g.rowscale ? g.rowscale + (long)b * g.strideRS : nullptr;
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int jj = 0; jj < WN; ++jj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm0 + i * 16 + acc_row(lane, r);
        const int gn = n0 + wn0 + jj * 16 + acc_col(lane, r);
        if (gm < g.M && gn < g.N) {
          double v = g.alpha * acc[i][jj][r];
          if (RS) v *= RS[gm];
          if (FSO) v *= (S[gm] > 0) ? rpos : rneg;
          const long o = (long)gm * g.ldc + gn;
          if (g.beta != 0.0) {
            const double cin = g.c_ident ? (gm == gn ? 1.0 : 0.0) : (gm < g.c_zero_rows ? 0.0 : C[o]);
            v += g.beta * cin;
          }
          C[o] = v;
        }
      }
}

template <int WM, int WN, int GM, int GN, int TK>
static int run(const GemmArgs& a, bool ta, bool tb, hipStream_t st) {
  constexpr int TM = 16 * WM * GM, TN = 16 * WN * GN;
  const int ntm = (a.M + TM - 1) / TM, ntn = (a.N + TN - 1) / TN;
  const long groups = ((long)a.batch + NXCD - 1) / NXCD * NXCD * ntm * ntn;
  dim3 grid((unsigned)groups);
  dim3 block(64 * GM * GN);
  if ((a.a_upper || a.S) && (ta || tb)) {
    set_error("triangular or field-scaled GEMMs are only supported untransposed");
    return SLQ_ERR_ARG;
  }
  if (a.brow && !a.a_upper) {
    set_error("a row gather of B is only supported with a triangular A");
    return SLQ_ERR_ARG;
  }
  if (a.a_upper && a.S) {
    set_error("a GEMM is either triangular or field-scaled");
    return SLQ_ERR_ARG;
  }
  if (a.a_upper) {
    const size_t lds = a.brow ? sizeof(int) * (size_t)a.K : 0;
    k_gemm<WM, WN, GM, GN, TK, false, false, 1><<<grid, block, lds, st>>>(a, ntm, ntn);
  } else if (a.S && a.s_out) {
    if (a.M != a.K) {
      set_error("output-row field scaling needs M == K");
      return SLQ_ERR_ARG;
    }
    k_gemm<WM, WN, GM, GN, TK, false, false, 3><<<grid, block, 0, st>>>(a, ntm, ntn);
  } else if (a.S) {
    k_gemm<WM, WN, GM, GN, TK, false, false, 2><<<grid, block, 0, st>>>(a, ntm, ntn);
  } else if (!ta && !tb) {
    k_gemm<WM, WN, GM, GN, TK, false, false, 0><<<grid, block, 0, st>>>(a, ntm, ntn);
  } else if (ta && !tb) {
    k_gemm<WM, WN, GM, GN, TK, true, false, 0><<<grid, block, 0, st>>>(a, ntm, ntn);
  } else if (!ta && tb) {
    k_gemm<WM, WN, GM, GN, TK, false, true, 0><<<grid, block, 0, st>>>(a, ntm, ntn);
  } else {
    k_gemm<WM, WN, GM, GN, TK, true, true, 0><<<grid, block, 0, st>>>(a, ntm, ntn);
  }
  SLQ_LAUNCHED();
  return SLQ_OK;
}

// Tile configurations of the FP64 GEMM (index = GemmCfg).
int launch_gemm_cfg(const GemmArgs& a, bool ta, bool tb, int cfg, hipStream_t st) {
  if (a.batch <= 0 || a.M <= 0 || a.N <= 0) return SLQ_OK;
  switch (cfg) {
    case GEMM_16: return run<1, 1, 1, 1, 16>(a, ta, tb, st);
    case GEMM_32x64: return run<2, 1, 1, 4, 16>(a, ta, tb, st);
    case GEMM_128: return run<4, 4, 2, 2, 8>(a, ta, tb, st);
    case GEMM_96: return run<3, 3, 2, 2, 8>(a, ta, tb, st);
    case GEMM_80_K4: return run<5, 1, 1, 5, 4>(a, ta, tb, st);
    case GEMM_80_K8: return run<5, 1, 1, 5, 8>(a, ta, tb, st);
    case GEMM_160x80: return run<5, 1, 2, 5, 8>(a, ta, tb, st);
    case GEMM_64: return run<2, 2, 2, 2, 8>(a, ta, tb, st);
    case GEMM_48: return run<3, 1, 1, 3, 8>(a, ta, tb, st);
    case GEMM_64x128: return run<2, 2, 2, 4, 8>(a, ta, tb, st);
    case GEMM_128x64: return run<2, 2, 4, 2, 8>(a, ta, tb, st);
    case GEMM_16x64: return run<1, 1, 1, 4, 16>(a, ta, tb, st);
    case GEMM_128x16: return run<2, 1, 4, 1, 8>(a, ta, tb, st);
    case GEMM_32x64_K32: return run<2, 1, 1, 4, 32>(a, ta, tb, st);
    case GEMM_16x64_K32: return run<1, 1, 1, 4, 32>(a, ta, tb, st);
    case GEMM_BIG: return gemm_big_ok(a, ta, tb) ? launch_gemm_big(a, ta, st) : run<2, 2, 4, 2, 8>(a, ta, tb, st);
    case GEMM_LEAN: return gemm_lean_ok(a, ta, tb) ? launch_gemm_lean(a, st) : run<2, 2, 4, 2, 8>(a, ta, tb, st);
    default:
      set_error("unknown GEMM tile configuration");
      return SLQ_ERR_ARG;
  }
}

// Default tile choice: thin panels get 32 x 64 tiles; otherwise the largest
// square tile that divides both M and N, else 64 x 64 with ragged edges.
// K is staged 4-8 deep: the small LDS footprint keeps several workgroups
// resident per CU, which hides the memory latency better than deeper stages
// (400 x 400 chain, 80 x 80 tiles: 16 deep 21.5, 8 deep 28.1, 4 deep
// 31.7 TFLOP/s).
int default_gemm(int M, int N) {
  auto divides = [&](int t) { return M % t == 0 && N % t == 0; };
  if (M <= 16 && N <= 16) return GEMM_16;
  if (M <= 32) return GEMM_32x64;
  if (M >= 128 && divides(128)) return GEMM_128;
  if (M >= 96 && divides(96)) return GEMM_96;
  if (M >= 80 && divides(80)) return GEMM_80_K4;
  if (M >= 64 && divides(64)) return GEMM_64;
  if (M >= 48 && divides(48)) return GEMM_48;
  return GEMM_64;
}

// Time every candidate tile shape of the dense FP64 chain GEMM, X <- E diag(d) X,
// on the plan's own buffers (Xa <- identity, spins all +1) and keep the fastest.
int tune_chain_gemm(Plan& p, int batch, hipStream_t st, float* best_ms_out) {
  const int N = p.n;
  std::vector<int> cands;
  if (N <= 32)
    cands = {GEMM_16, GEMM_32x64, GEMM_64};
  else
    cands = {GEMM_128, GEMM_96, GEMM_80_K4, GEMM_80_K8, GEMM_160x80, GEMM_64, GEMM_48, GEMM_128x64, GEMM_64x128};
  const long NN = (long)N * N;
  SLQ_TRY(launch_set_identity(p, batch, p.Xa, st));
  SLQ_TRY(fill_i32((int32_t*)p.s_work, (long)batch * p.L * N / 4, 0x01010101, st));
  GemmArgs a{};
  a.M = N;
  a.N = N;
  a.K = N;
  a.A = p.E;
  a.lda = N;
  a.B = p.Xa;
  a.ldb = N;
  a.strideB = NN;
  a.C = p.Xb;
  a.ldc = N;
  a.strideC = NN;
  a.S = p.s_work;
  a.strideS = (long)p.L * N;
  a.consts = p.consts;
  a.alpha = 1.0;
  a.batch = batch;
  hipEvent_t e0, e1;
  SLQ_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    set_error("hipEventCreate failed");
    return SLQ_ERR_DEVICE;
  }
  int best = default_gemm(N, N), rc = SLQ_OK;
  float best_ms = 1e30f;
  for (int cfg : cands) {
    if ((rc = launch_gemm_cfg(a, false, false, cfg, st)) != SLQ_OK) break;
    if (hipEventRecord(e0, st) != hipSuccess) rc = SLQ_ERR_DEVICE;
    for (int r = 0; r < 3 && rc == SLQ_OK; ++r) rc = launch_gemm_cfg(a, false, false, cfg, st);
    float ms = 0.f;
    if (rc == SLQ_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = SLQ_ERR_DEVICE;
    if (rc != SLQ_OK) break;
    if (ms < best_ms) {
      best_ms = ms;
      best = cfg;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != SLQ_OK) {
    if (rc == SLQ_ERR_DEVICE) set_error("timing the chain GEMM tile shapes failed");
    return rc;
  }
  p.gemm_cfg = best;
  if (best_ms_out) *best_ms_out = best_ms;
  return SLQ_OK;
}

int launch_gemm(const GemmArgs& a, bool ta, bool tb, hipStream_t st) {
  int cfg = -1;
  if (a.cfg >= 0) cfg = a.cfg;
  // the triangular product of the stabilisation (400^3, 512 fields: 0.96 ms
  // on 64 x 128 tiles against 1.01 ms on 80 x 80)
  if (cfg < 0 && a.a_upper && a.M >= 64) cfg = GEMM_64x128;
  if (cfg < 0) cfg = default_gemm(a.M, a.N);
  return launch_gemm_cfg(a, ta, tb, cfg, st);
}

}  // namespace slq
