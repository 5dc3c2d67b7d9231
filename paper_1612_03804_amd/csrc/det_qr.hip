// Final step of a weight-only evaluation on the matrix cores: log|det(1 + U D V)|
// and its sign from a Householder QR of M (no G).
//
// With D_b = max(D, 1) and D_s = min(D, 1),
//     1 + U D V = U D_b M,   M = D_b^{-1} U^T + D_s V,
// so det(1 + B_L...B_1) (the fermion determinant of Eq. 1; the paper's
// "N^3 from calculating the determinant") is det(U) prod(D_b) det(M).  M is
// well conditioned (the large scales sit in D_b^{-1} <= 1, the small ones in
// D_s <= 1), so an orthogonal factorisation M Pi = Q R needs no care beyond
// that of the stabilisation itself: det M = det Q prod(R_ii) sign(Pi), with
// det Q = (-1)^(reflectors with tau != 0).  The R-only blocked QR of the
// stabilisation (panels in registers, compact-WY trailing updates on FP64
// MFMA, no explicit Q) spreads every field over many workgroups, where an LU
// in one workgroup per field is bound by a single CU's bandwidth.
#include "slq_internal.h"

namespace slq {

constexpr int BM_T = 64;         // tile edge of the M build
constexpr int BM_THREADS = 256;

// M[k][j] = U[j][k] / max(D[k], 1) + min(D[k], 1) V[k][j], tiled through LDS
// so that U is read along its rows and M written along its rows.
__global__ __launch_bounds__(BM_THREADS) void k_build_m(int N, const double* __restrict__ Uall,
                                                        const double* __restrict__ Dall,
                                                        const double* __restrict__ Vall, double* __restrict__ Mall) {
  __shared__ double tile[BM_T][BM_T + 1];
  const long b = blockIdx.z;
  const long NN = (long)N * N;
  const double* U = Uall + b * NN;
  const double* V = Vall + b * NN;
  const double* D = Dall + b * N;
  double* M = Mall + b * NN;
  const int kb = blockIdx.x * BM_T, jb = blockIdx.y * BM_T;
  const int tx = threadIdx.x % BM_T, ty = threadIdx.x / BM_T;  // 64 x 4
  // U rows jb.., columns kb..: tile[j][k]
  for (int r = ty; r < BM_T; r += BM_THREADS / BM_T) {
    const int j = jb + r, k = kb + tx;
    tile[r][tx] = (j < N && k < N) ? U[(long)j * N + k] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < BM_T; r += BM_THREADS / BM_T) {
    const int k = kb + r, j = jb + tx;
    if (k < N && j < N) {
      const double d = D[k];
      M[(long)k * N + j] = tile[tx][r] / fmax(d, 1.0) + fmin(d, 1.0) * V[(long)k * N + j];
    }
  }
}

// One workgroup per field: log|det| and sign from the chain's D and
// reflector count, and the QR of M (|R_ii| in DM, R in W, the column
// permutation perm and its reflector count nrefM).
constexpr int DQ_THREADS = 256;

__global__ __launch_bounds__(DQ_THREADS) void k_det_qr(int N, const double* __restrict__ Dall,
                                                       const int32_t* __restrict__ nref,
                                                       const double* __restrict__ DMall, const double* __restrict__ Wall,
                                                       const int32_t* __restrict__ permall,
                                                       const int32_t* __restrict__ nrefM, double* logabs,
                                                       int8_t* sign, int32_t* status) {
  __shared__ double red[DQ_THREADS / 64];
  __shared__ int redi[DQ_THREADS / 64][3];
  __shared__ unsigned char seen[2432];
  __shared__ int pperm;
  const long b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* D = Dall + b * N;
  const double* DM = DMall + b * N;
  const double* W = Wall + b * (long)N * N;
  const int32_t* perm = permall + b * N;
  double ls = 0.0;
  int neg = 0, zero = 0, bad = 0;
  for (int i = tid; i < N; i += DQ_THREADS) {
    const double dm = DM[i];
    ls += log(fmax(D[i], 1.0)) + log(dm);
    neg ^= W[(long)i * N + i] < 0.0;
    zero |= dm == 0.0;
    bad |= !(dm < INFINITY);  // NaN or +inf
    seen[i] = 0;
  }
  ls = wave_sum(ls);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    neg ^= __shfl_xor(neg, o, 64);
    zero |= __shfl_xor(zero, o, 64);
    bad |= __shfl_xor(bad, o, 64);
  }
  if (lane == 0) {
    red[wave] = ls;
    redi[wave][0] = neg;
    redi[wave][1] = zero;
    redi[wave][2] = bad;
  }
  __syncthreads();
  if (tid == 0) {
    // parity of the column permutation: N minus the number of its cycles
    int cycles = 0;
    for (int i = 0; i < N; ++i) {
      if (seen[i]) continue;
      ++cycles;
      for (int j = i; !seen[j]; j = perm[j]) seen[j] = 1;
    }
    pperm = (N - cycles) & 1;
    double tot = 0.0;
    int par = (nref[b] & 1) ^ (nrefM[b] & 1) ^ pperm, sing = 0, nonfin = 0;
    for (int w = 0; w < DQ_THREADS / 64; ++w) {
      tot += red[w];
      par ^= redi[w][0];
      sing |= redi[w][1];
      nonfin |= redi[w][2];
    }
    if (nonfin || (!sing && !isfinite(tot))) {
      if (status) status[b] |= SLQ_ST_NONFINITE;
    } else if (sing) {
      if (status) status[b] |= SLQ_ST_SINGULAR;
    }
    logabs[b] = sing && !nonfin ? -INFINITY : tot;
    sign[b] = sing ? 0 : (par ? -1 : 1);
  }
}

// True when the plan's buffers that the QR of M uses are free of f.
static bool det_qr_usable(const Plan& p, const UdvRef& f) {
  if (p.n <= 64) return false;  // one-workgroup QR and LU are already one launch per field
  const double* used[] = {p.Xa, p.Xb, p.W, p.Vt};
  for (const double* u : used)
    if (f.U == u || f.V == u || f.D == u) return false;
  return true;
}

int launch_det_qr(Plan& p, int batch, const UdvRef& f, double* logabs, int8_t* sign, int32_t* status,
                  hipStream_t st) {
  const int N = p.n;
  const dim3 grid((N + BM_T - 1) / BM_T, (N + BM_T - 1) / BM_T, batch);
  k_build_m<<<grid, BM_THREADS, 0, st>>>(N, f.U, f.D, f.V, p.Xa);
  SLQ_LAUNCHED();
  // QR of M with unit column scales: D of the factorisation in Vt (first N
  // doubles per field), its reflector count and status in the plan's spares
  double* DM = p.Vt;
  SLQ_TRY(fill_f64(DM, (long)batch * N, 1.0, st));
  const UdvRef m{nullptr, DM, nullptr, p.nref2};
  SLQ_TRY(launch_qr_blocked(p, batch, p.Xa, m, p.status2, st, nullptr, false));
  k_det_qr<<<batch, DQ_THREADS, 0, st>>>(N, f.D, f.nref, DM, p.W, p.perm, p.nref2, logabs, sign, status);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

bool use_det_qr(const Plan& p, const UdvRef& f) { return det_qr_usable(p, f); }

}  // namespace slq
