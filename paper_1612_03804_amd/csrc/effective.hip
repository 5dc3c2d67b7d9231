// Effective bosonic action and the moves, features, acceptance and fit built
// on it ("Formalism of SLDQMC", Eqs. 2-4, and the R^2 score of "Results").
//
//   S_eff(s) = c0 + sum_k lambda_k F_k(s),   F_k = 1/2 sum_x s_x h_k(x),
//   h_k((i, l)) = sum_{delta in shell r_k} s_{i+delta, l+dl_k} + s_{i+delta, l-dl_k}  (dl_k > 0)
//               = sum_{delta in shell r_k} s_{i+delta, l}                             (dl_k = 0)
//
// A flip of x changes S_eff by dS = -2 s_x sum_k lambda_k h_k(x).  Moves act
// on colour classes (one slice, one colour of the greedy colouring of the
// dl = 0 coupling graph), so all sites of a class are updated at once without
// touching each other's partners; drawing the class at random keeps the
// effective chain reversible for exp(S_eff), which the cumulative-update
// acceptance of Eq. 4 relies on.
#include <algorithm>
#include <cstring>
#include <new>
#include <set>
#include <vector>

#include "slq_internal.h"

namespace slq {


constexpr int MAX_TERMS = 64;
constexpr int MAX_SHELL = 5;

// Offsets of shells 0..5, ordered by squared length 0, 1, 2, 4, 5, 8.
static const int kShellOff[MAX_SHELL + 2] = {0, 1, 5, 9, 13, 21, 25};
static const int kShellDxy[25][2] = {
    {0, 0},                                              // 0
    {1, 0},  {-1, 0}, {0, 1},  {0, -1},                  // 1
    {1, 1},  {1, -1}, {-1, 1}, {-1, -1},                 // 2
    {2, 0},  {-2, 0}, {0, 2},  {0, -2},                  // 3
    {2, 1},  {2, -1}, {-2, 1}, {-2, -1}, {1, 2}, {1, -2}, {-1, 2}, {-1, -2},  // 4
    {2, 2},  {2, -2}, {-2, 2}, {-2, -2}};                // 5

EffDev eff_dev_view(const Plan& p, const Eff& e) {
  EffDev d;
  d.lx = p.m.lx;
  d.ly = p.m.ly;
  d.L = p.L;
  d.N = p.n;
  d.n_terms = e.n_terms;
  d.n_colours = e.n_colours;
  d.n_classes = e.n_classes;
  d.terms = e.d_terms;
  d.theta = e.d_theta;
  d.col_sites = e.d_col_sites;
  d.col_off = e.d_col_off;
  d.shell_off = e.d_shell_off;
  d.shell_dxy = e.d_shell_dxy;
  d.n_pairs = e.n_pairs;
  d.pairs = e.d_pairs;
  d.n_uoff = e.n_uoff;
  d.uoff = e.d_uoff;
  return d;
}

// ------------------------------------------------------------ moves ----
__global__ __launch_bounds__(256) void k_eff_sweep(EffDev d, int8_t* s_all, int n_moves, uint64_t seed,
                                                   uint64_t step, uint64_t chain0, int64_t* accepts, double* dS_out) {
  __shared__ double redd[4];
  __shared__ long long redi[4];
  const int b = blockIdx.x;
  int8_t* s = s_all + (long)b * d.L * d.N;
  const uint64_t chain = chain0 + b;
  long long acc = 0;
  double dsum = 0.0;
  for (int mv = 0; mv < n_moves; ++mv) {
    const uint32_t cls = philox_below((uint32_t)d.n_classes, 0, (uint64_t)mv, step, chain, seed, TAG_EFFECTIVE);
    const int colour = (int)(cls % d.n_colours);
    const int l = (int)(cls / d.n_colours);  // 0-based slice
    const int beg = d.col_off[colour], end = d.col_off[colour + 1];
    for (int t = beg + threadIdx.x; t < end; t += blockDim.x) {
      const int i = d.col_sites[t];
      double hs = 0.0;
      for (int k = 0; k < d.n_terms; ++k) hs += d.theta[1 + k] * (double)local_field_dev(d, s, k, i, l);
      const double sx = (double)s[(long)l * d.N + i];
      const double dS = -2.0 * sx * hs;
      const double u = philox_uniform((uint64_t)(1 + (long)l * d.N + i), (uint64_t)mv, step, chain, seed,
                                      TAG_EFFECTIVE);
      if (u < exp(dS)) {
        s[(long)l * d.N + i] = (int8_t)(-s[(long)l * d.N + i]);
        ++acc;
        dsum += dS;
      }
    }
    __syncthreads();
  }
  dsum = wave_sum(dsum);
  long long a2 = acc;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a2 += __shfl_xor(a2, o, 64);
  if ((threadIdx.x & 63) == 0) {
    redd[threadIdx.x >> 6] = dsum;
    redi[threadIdx.x >> 6] = a2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (accepts) accepts[b] = redi[0] + redi[1] + redi[2] + redi[3];
    if (dS_out) dS_out[b] = ((redd[0] + redd[1]) + redd[2]) + redd[3];
  }
}

// The same moves with the field, the couplings and the flattened partner
// list in LDS.  Four lanes share a site, each summing every fourth partner;
// a quad reduction joins them and the first lane draws and flips.
constexpr int EFF_THREADS = 512;
constexpr int EFF_LPS = 4;  // lanes per site

__device__ __forceinline__ int wrap2(int v, int n) {  // v in [-2n, 3n)
  if (v < 0) v += n;
  if (v < 0) v += n;
  if (v >= n) v -= n;
  if (v >= n) v -= n;
  return v;
}

// BITS: the field as one bit per spin (1 for s = +1) in 32-bit LDS words,
// flipped with an LDS atomic xor (sites of a class can share a word); the
// 48x48, L = 100 field takes 28.8 KB so, against 230 KB as bytes.
template <bool BITS>
__global__ __launch_bounds__(EFF_THREADS) void k_eff_sweep_lds(EffDev d, int8_t* s_all, int n_moves, uint64_t seed,
                                                                uint64_t step, uint64_t chain0, int64_t* accepts,
                                                                double* dS_out) {
  extern __shared__ double sm[];
  __shared__ double redd[EFF_THREADS / 64];
  __shared__ long long redi[EFF_THREADS / 64];
  __shared__ double one_body;
  const int np = d.n_pairs, N = d.N, L = d.L, lx = d.lx, ly = d.ly;
  double* lam = sm;                            // [np]
  int32_t* pr = (int32_t*)(lam + np);          // [np]: u N | (dt + 2048) << 16
  int16_t* spart = (int16_t*)(pr + np);        // [n_uoff][N]: partner site of each site under offset u
  int16_t* csite = spart + d.n_uoff * N;       // [N] sites by colour
  int16_t* coff = csite + N;                   // [n_colours + 1]
  int8_t* f = (int8_t*)(coff + d.n_colours + 1); // [L][N] bytes, or (BITS) [ceil(L N / 32)] words:
  uint32_t* fw = (uint32_t*)(((uintptr_t)f + 3) & ~(uintptr_t)3);
  const int b = blockIdx.x, tid = threadIdx.x;
  int8_t* s = s_all + (long)b * L * N;
  const uint64_t chain = chain0 + b;
  for (int p = tid; p < np; p += EFF_THREADS) {
    const int32_t e = d.pairs[p];
    pr[p] = (e & 255) * N | (((e >> 8) & 4095) << 16);
    lam[p] = d.theta[1 + (e >> 20)];
  }
  for (int i = tid; i < N; i += EFF_THREADS) csite[i] = (int16_t)d.col_sites[i];
  for (int c = tid; c <= d.n_colours; c += EFF_THREADS) coff[c] = (int16_t)d.col_off[c];
  for (int idx = tid; idx < d.n_uoff * N; idx += EFF_THREADS) {
    const int u = idx / N, i = idx % N;
    const int xx = wrap2(i % lx + d.uoff[2 * u], lx), yy = wrap2(i / lx + d.uoff[2 * u + 1], ly);
    spart[idx] = (int16_t)(xx + lx * yy);
  }
  if (tid == 0) {
    double h = 0.0;
    for (int k = 0; k < d.n_terms; ++k)
      if (d.terms[2 * k] == 0 && d.terms[2 * k + 1] == 0) h += d.theta[1 + k];
    one_body = h;
  }
  const long LN = (long)L * N;
  if constexpr (BITS) {
    for (long w = tid; w < (LN + 31) / 32; w += EFF_THREADS) {
      uint32_t v = 0;
      for (int k = 0; k < 32 && 32 * w + k < LN; ++k) v |= (uint32_t)(s[32 * w + k] > 0) << k;
      fw[w] = v;
    }
  } else {
    for (long i = tid; i < LN; i += EFF_THREADS) f[i] = s[i];
  }
  __syncthreads();
  auto spin = [&](int q) -> int {  // s at flat index q = l N + i, as +-1
    if constexpr (BITS)
      return (int)((fw[q >> 5] >> (q & 31)) & 1u) * 2 - 1;
    else
      return f[q];
  };
  const int sub = tid & (EFF_LPS - 1), slot = tid / EFF_LPS, nslot = EFF_THREADS / EFF_LPS;
  const double h1 = one_body;
  long long acc = 0;
  double dsum = 0.0;
  for (int mv = 0; mv < n_moves; ++mv) {
    const uint32_t cls = philox_below((uint32_t)d.n_classes, 0, (uint64_t)mv, step, chain, seed, TAG_EFFECTIVE);
    const int colour = (int)(cls % d.n_colours);
    const int l = (int)(cls / d.n_colours);  // 0-based slice
    const int beg = coff[colour], end = coff[colour + 1];
    for (int t = beg + slot; t < end; t += nslot) {  // the lanes of a group share t
      const int i = csite[t];
      const int16_t* sp_i = spart + i;
      // partners p = sub, sub + 4, ... four at a time: their LDS reads are in
      // flight together (the sum keeps the order p = sub, sub + 4, ...)
      double hs = 0.0;
      constexpr int32_t kSelf = 2048 << 16;  // offset 0 of slice l: a valid address, weight 0
      for (int p0 = sub; p0 < np; p0 += 4 * EFF_LPS) {
        int32_t e[4];
        double w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int p = p0 + EFF_LPS * u;
          e[u] = p < np ? pr[p] : kSelf;
          w[u] = p < np ? lam[p] : 0.0;
        }
        double sp[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          int ll = l + (e[u] >> 16) - 2048;
          if (ll < 0) ll += L;
          if (ll >= L) ll -= L;
          sp[u] = (double)spin(__umul24(ll, N) + sp_i[e[u] & 0xffff]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) hs += w[u] * sp[u];
      }
      hs += dpp_move<DPP_QUAD_XOR1>(hs);
      hs += dpp_move<DPP_QUAD_XOR2>(hs);
      if (sub == 0) {
        const int q = l * N + i;
        const int sv = spin(q);
        const double dS = -2.0 * (double)sv * (h1 + hs);
        const double u = philox_uniform((uint64_t)(1 + (long)l * N + i), (uint64_t)mv, step, chain, seed,
                                        TAG_EFFECTIVE);
        if (u < exp(dS)) {
          if constexpr (BITS)
            atomicXor(&fw[q >> 5], 1u << (q & 31));
          else
            f[q] = (int8_t)(-sv);
          ++acc;
          dsum += dS;
        }
      }
    }
    __syncthreads();
  }
  for (long i = tid; i < LN; i += EFF_THREADS) s[i] = (int8_t)spin((int)i);
  dsum = wave_sum(dsum);
  const double a2 = wave_sum((double)acc);  // exact: counts stay far below 2^53
  if ((tid & 63) == 0) {
    redd[tid >> 6] = dsum;
    redi[tid >> 6] = (long long)a2;
  }
  __syncthreads();
  if (tid == 0) {
    long long at = 0;
    double ds = 0.0;
    for (int w = 0; w < EFF_THREADS / 64; ++w) {
      at += redi[w];
      ds += redd[w];
    }
    if (accepts) accepts[b] = at;
    if (dS_out) dS_out[b] = ds;
  }
}

static size_t eff_lds_bytes(const Plan& p, const Eff& e, bool bits) {
  const size_t field = bits ? 4 + 4 * (((size_t)p.L * p.n + 31) / 32) : (size_t)p.L * p.n;
  return (size_t)e.n_pairs * (sizeof(double) + sizeof(int32_t)) +
         ((size_t)e.n_uoff * p.n + p.n + e.n_colours + 1) * sizeof(int16_t) + field;
}

int launch_eff_sweep(Plan& p, const Eff& e, int batch, int8_t* s, int n_moves, uint64_t seed, uint64_t step,
                     uint64_t chain0, int64_t* accepts, double* dS, hipStream_t st) {
  if (batch <= 0) return SLQ_OK;
  if (e.net_on) return launch_eff_sweep_net(p, e, batch, s, n_moves, seed, step, chain0, accepts, dS, st);
  // the field in LDS as bytes where it fits, else as bits (the 48x48, L = 100
  // field: 28.8 KB), else the kernel that reads it from global memory
  const size_t lds = eff_lds_bytes(p, e, false), ldsb = eff_lds_bytes(p, e, true);
  const bool lds_ok = e.d_pairs && p.L <= 4094;
  if (lds_ok && lds <= 150 * 1024) {
    allow_max_lds((const void*)k_eff_sweep_lds<false>);
    k_eff_sweep_lds<false><<<batch, EFF_THREADS, lds, st>>>(eff_dev_view(p, e), s, n_moves, seed, step, chain0,
                                                            accepts, dS);
  } else if (lds_ok && ldsb <= 150 * 1024) {
    allow_max_lds((const void*)k_eff_sweep_lds<true>);
    k_eff_sweep_lds<true><<<batch, EFF_THREADS, ldsb, st>>>(eff_dev_view(p, e), s, n_moves, seed, step, chain0,
                                                            accepts, dS);
  } else {
    k_eff_sweep<<<batch, 256, 0, st>>>(eff_dev_view(p, e), s, n_moves, seed, step, chain0, accepts, dS);
  }
  SLQ_LAUNCHED();
  return SLQ_OK;
}

// --------------------------------------------------------- features ----
// F[b][k] = 1/2 sum_x s_x h_k(x), sum_x s_x for the one-body term; integer
// sums, exact.
__global__ __launch_bounds__(256) void k_features(EffDev d, const int8_t* s_all, double* F) {
  __shared__ long long acc[MAX_TERMS];
  const long b = blockIdx.x;
  const int8_t* s = s_all + b * d.L * d.N;
  for (int k = threadIdx.x; k < d.n_terms; k += blockDim.x) acc[k] = 0;
  __syncthreads();
  const long total = (long)d.L * d.N;
  for (int k = 0; k < d.n_terms; ++k) {
    long long part = 0;
    for (long x = threadIdx.x; x < total; x += blockDim.x) {
      const int l = (int)(x / d.N), i = (int)(x % d.N);
      part += (long long)s[x] * local_field_dev(d, s, k, i, l);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd((unsigned long long*)&acc[k], (unsigned long long)part);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < d.n_terms; k += blockDim.x) {
    const bool one_body = d.terms[2 * k] == 0 && d.terms[2 * k + 1] == 0;
    F[b * d.n_terms + k] = (one_body ? 1.0 : 0.5) * (double)acc[k];
  }
}

// The same features from per-site bit strings of the field along imaginary
// time: with bit l of B_i set when s_{i,l} = -1,
//     sum_l s_{i,l} s_{j,l+t} = L - 2 popcount(B_i xor B_j rotated by t),
// and, the shells being symmetric under delta -> -delta,
//     F_(r,dl) = sum_{delta in shell r} sum_{i,l} s_{i,l} s_{i+delta, l+dl}   (dl > 0),
//     F_(r,0)  = 1/2 of the same sum with dl = 0,   F_(0,0) = sum_{i,l} s_{i,l}.
// Each site keeps B twice over (2L bits) so a rotation is a shifted read.
constexpr int FEAT_THREADS = 512;

__device__ __forceinline__ uint64_t bits_window(const uint64_t* D, int t, int w) {  // bits t + 64 w ...
  const int q = (t >> 6) + w, r = t & 63;
  return r == 0 ? D[q] : (D[q] >> r) | (D[q + 1] << (64 - r));
}

__global__ __launch_bounds__(FEAT_THREADS) void k_features_bits(EffDev d, const int8_t* s_all, double* F) {
  extern __shared__ uint64_t bits[];  // [N][W2]
  __shared__ double part[FEAT_THREADS / 64][MAX_TERMS];
  const int N = d.N, L = d.L, lx = d.lx, ly = d.ly, K = d.n_terms;
  const int W = (L + 63) / 64, W2 = (2 * L + 63) / 64 + 1;
  const uint64_t last = (L % 64) ? ((1ull << (L % 64)) - 1) : ~0ull;
  const long b = blockIdx.x;
  const int8_t* s = s_all + b * L * N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < N; i += FEAT_THREADS) {
    uint64_t* D = bits + (long)i * W2;
    for (int w = 0; w < W2; ++w) {
      uint64_t v = 0;
      for (int t = 0; t < 64; ++t) {
        const int l = 64 * w + t;
        if (l < 2 * L && s[(long)(l < L ? l : l - L) * N + i] < 0) v |= 1ull << t;
      }
      D[w] = v;
    }
  }
  __syncthreads();
  for (int k = 0; k < K; ++k) {
    const int r = d.terms[2 * k], dl = d.terms[2 * k + 1];
    long long acc = 0;
    for (int i = tid; i < N; i += FEAT_THREADS) {
      const uint64_t* Di = bits + (long)i * W2;
      if (r == 0 && dl == 0) {
        int ones = 0;
        for (int w = 0; w < W; ++w) ones += __popcll(Di[w] & (w == W - 1 ? last : ~0ull));
        acc += L - 2 * ones;
        continue;
      }
      const int x = i % lx, y = i / lx;
      for (int o = d.shell_off[r]; o < d.shell_off[r + 1]; ++o) {
        int xx = x + d.shell_dxy[2 * o], yy = y + d.shell_dxy[2 * o + 1];
        xx = ((xx % lx) + lx) % lx;
        yy = ((yy % ly) + ly) % ly;
        const uint64_t* Dj = bits + (long)(xx + lx * yy) * W2;
        int diff = 0;
        for (int w = 0; w < W; ++w)
          diff += __popcll((Di[w] ^ bits_window(Dj, dl, w)) & (w == W - 1 ? last : ~0ull));
        acc += L - 2 * diff;
      }
    }
    const double tot = wave_sum((double)acc);  // exact integers
    if (lane == 0) part[wave][k] = tot;
  }
  __syncthreads();
  for (int k = tid; k < K; k += FEAT_THREADS) {
    double t = 0.0;
    for (int w = 0; w < FEAT_THREADS / 64; ++w) t += part[w][k];
    const int r = d.terms[2 * k], dl = d.terms[2 * k + 1];
    F[b * K + k] = (dl == 0 && r != 0) ? 0.5 * t : t;
  }
}

int launch_features(Plan& p, const Eff& e, long count, const int8_t* s, double* F, hipStream_t st) {
  if (count <= 0) return SLQ_OK;
  const size_t lds = (size_t)p.n * ((2 * p.L + 63) / 64 + 1) * sizeof(uint64_t);
  if (lds <= 120 * 1024) {
    allow_max_lds((const void*)k_features_bits);
    k_features_bits<<<(unsigned)count, FEAT_THREADS, lds, st>>>(eff_dev_view(p, e), s, F);
  } else {
    k_features<<<(unsigned)count, 256, 0, st>>>(eff_dev_view(p, e), s, F);
  }
  SLQ_LAUNCHED();
  return SLQ_OK;
}

// ----------------------------------------------------------- accept ----
// Eq. 4: logA = [ln|W(s')| - ln|W(s)|] - [S_eff(s') - S_eff(s)]
__global__ __launch_bounds__(256) void k_accept(EffDev d, int8_t* s_all, const int8_t* sp_all, double* logabs,
                                                int8_t* sign, const double* new_logabs, const int8_t* new_sign,
                                                const double* F_old, const double* F_new, const double* Sn_old,
                                                const double* Sn_new, uint64_t seed, uint64_t step, uint64_t chain0,
                                                int8_t* accepted, double* logA) {
  __shared__ int take;
  const int b = blockIdx.x;
  if (threadIdx.x == 0) {
    double dS = 0.0;
    for (int k = 0; k < d.n_terms; ++k)
      dS += d.theta[1 + k] * (F_new[(long)b * d.n_terms + k] - F_old[(long)b * d.n_terms + k]);
    if (Sn_old) dS += Sn_new[b] - Sn_old[b];  // learned part of the action
    const double la = (new_logabs[b] - logabs[b]) - dS;
    const double u = philox_uniform(0, 0, step, chain0 + b, seed, TAG_CUMULATIVE);
    const double lu = (u == 0.0) ? -INFINITY : log(u);
    const bool ok = new_sign[b] != 0 && lu < fmin(0.0, la);
    take = ok;
    if (accepted) accepted[b] = ok ? 1 : 0;
    if (logA) logA[b] = la;
    if (ok) {
      logabs[b] = new_logabs[b];
      sign[b] = new_sign[b];
    }
  }
  __syncthreads();
  if (take) {
    const long total = (long)d.L * d.N;
    for (long x = threadIdx.x; x < total; x += blockDim.x) s_all[b * total + x] = sp_all[b * total + x];
  }
}

int launch_accept(Plan& p, const Eff& e, int batch, int8_t* s, const int8_t* sprop, double* logabs, int8_t* sign,
                  const double* new_logabs, const int8_t* new_sign, const double* F_old, const double* F_new,
                  const double* Sn_old, const double* Sn_new, uint64_t seed, uint64_t step, uint64_t chain0,
                  int8_t* accepted, double* logA, hipStream_t st) {
  if (batch <= 0) return SLQ_OK;
  k_accept<<<batch, 256, 0, st>>>(eff_dev_view(p, e), s, sprop, logabs, sign, new_logabs, new_sign, F_old, F_new,
                                  Sn_old, Sn_new, seed, step, chain0, accepted, logA);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

// -------------------------------------------------------------- fit ----
// OLS with an intercept on centred features: lambda = (Fc^T Fc)^{-1} Fc^T yc,
// c0 = ybar - Fbar . lambda; R^2 from the explicit residuals.  The samples
// arrive in chunks (their features computed into the plan's buffer one chunk
// at a time), so the sums are kept about a shift, the means of the first
// chunk (z = (F, y) - c):  sum (z_k - zbar_k)(z_l - zbar_l) =
// sum z_k z_l - (sum z_k)(sum z_l) / n, with small sums because the shift
// sits near the means.  Each sum has one owner thread that adds the rows in
// order: the result does not depend on the chunking's timing (deterministic).
constexpr int FIT_THREADS = 1024;
constexpr int FA_K1 = MAX_TERMS + 1;          // features and y
constexpr int FA_N = 0;                       // samples so far
constexpr int FA_SHIFT = 1;                   // [FA_K1]
constexpr int FA_SUM = FA_SHIFT + FA_K1;      // [FA_K1] sum of z
constexpr int FA_GRAM = FA_SUM + FA_K1;       // [FA_K1][FA_K1] sum of z_k z_l (k <= l)
constexpr int FA_YBAR = FA_GRAM + FA_K1 * FA_K1;
constexpr int FA_SSR = FA_YBAR + 1, FA_SST = FA_SSR + 1;
constexpr int FA_TOTAL = FA_SST + 1;
static_assert(FA_TOTAL <= FIT_ACC_DOUBLES, "fit accumulators exceed their buffer");

__global__ __launch_bounds__(FIT_THREADS) void k_fit_acc(int first, long rows, int K, const double* __restrict__ F,
                                                         const double* __restrict__ y, double* acc) {
  const int tid = threadIdx.x;
  auto z = [&](long i, int k) { return k < K ? F[i * K + k] : y[i]; };
  if (first) {
    for (int k = tid; k <= K; k += FIT_THREADS) {
      double s = 0.0;
      for (long i = 0; i < rows; ++i) s += z(i, k);
      acc[FA_SHIFT + k] = s / (double)rows;
      acc[FA_SUM + k] = 0.0;
    }
    for (int e = tid; e < FA_K1 * FA_K1; e += FIT_THREADS) acc[FA_GRAM + e] = 0.0;
    if (tid == 0) acc[FA_N] = 0.0;
    __syncthreads();
  }
  const double* c = acc + FA_SHIFT;
  const int npair = (K + 1) * (K + 2) / 2;
  for (int pr = tid; pr < npair + K + 1; pr += FIT_THREADS) {
    if (pr < npair) {
      int k1 = 0, rem = pr;
      while (rem >= K + 1 - k1) {
        rem -= K + 1 - k1;
        ++k1;
      }
      const int k2 = k1 + rem;
      double s = acc[FA_GRAM + k1 * FA_K1 + k2];
      for (long i = 0; i < rows; ++i) s += (z(i, k1) - c[k1]) * (z(i, k2) - c[k2]);
      acc[FA_GRAM + k1 * FA_K1 + k2] = s;
    } else {
      const int k = pr - npair;
      double s = acc[FA_SUM + k];
      for (long i = 0; i < rows; ++i) s += z(i, k) - c[k];
      acc[FA_SUM + k] = s;
    }
  }
  if (tid == 0) acc[FA_N] += (double)rows;
}

__global__ __launch_bounds__(FIT_THREADS) void k_fit_solve(int K, double* acc, double* theta) {
  __shared__ double mean[MAX_TERMS + 1];
  __shared__ double A[MAX_TERMS][MAX_TERMS + 1];
  __shared__ double rhs[MAX_TERMS];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const double n = acc[FA_N];
  const double* S = acc + FA_SUM;
  const double* Gm = acc + FA_GRAM;
  if (tid == 0) bad = 0;
  for (int k = tid; k <= K; k += FIT_THREADS) mean[k] = acc[FA_SHIFT + k] + S[k] / n;
  for (int e = tid; e < K * K; e += FIT_THREADS) {
    const int k1 = e / K, k2 = e % K, a = min(k1, k2), b = max(k1, k2);
    A[k1][k2] = Gm[a * FA_K1 + b] - S[a] * S[b] / n;
  }
  for (int k = tid; k < K; k += FIT_THREADS) rhs[k] = Gm[k * FA_K1 + K] - S[k] * S[K] / n;
  __syncthreads();
  // Cholesky A = L L^T in place (lower part)
  for (int j = 0; j < K; ++j) {
    if (tid == 0) {
      double djj = A[j][j];
      for (int m = 0; m < j; ++m) djj -= A[j][m] * A[j][m];
      if (!(djj > 0.0)) {
        bad = 1;
        djj = 1.0;
      }
      A[j][j] = sqrt(djj);
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < K; i += FIT_THREADS) {
      double v = A[i][j];
      for (int m = 0; m < j; ++m) v -= A[i][m] * A[j][m];
      A[i][j] = v / A[j][j];
    }
    __syncthreads();
  }
  if (tid == 0) {
    double zz[MAX_TERMS];
    for (int i = 0; i < K; ++i) {
      double v = rhs[i];
      for (int m = 0; m < i; ++m) v -= A[i][m] * zz[m];
      zz[i] = v / A[i][i];
    }
    for (int i = K - 1; i >= 0; --i) {
      double v = zz[i];
      for (int m = i + 1; m < K; ++m) v -= A[m][i] * rhs[m];
      rhs[i] = v / A[i][i];  // lambda_i (rhs reused, filled from the back)
    }
    double c0 = mean[K];
    for (int k = 0; k < K; ++k) c0 -= mean[k] * rhs[k];
    theta[0] = bad ? NAN : c0;
    for (int k = 0; k < K; ++k) theta[1 + k] = bad ? NAN : rhs[k];
    acc[FA_YBAR] = mean[K];
    acc[FA_SSR] = 0.0;
    acc[FA_SST] = 0.0;
  }
}

// explicit residuals of one chunk, added to the running sums in chunk order
__global__ __launch_bounds__(FIT_THREADS) void k_fit_resid(long rows, int K, const double* __restrict__ F,
                                                           const double* __restrict__ y, const double* theta,
                                                           double* acc) {
  __shared__ double red[2][FIT_THREADS / 64];
  const int tid = threadIdx.x;
  const double ybar = acc[FA_YBAR];
  double ssr = 0.0, sst = 0.0;
  for (long i = tid; i < rows; i += FIT_THREADS) {
    double yh = theta[0];
    for (int k = 0; k < K; ++k) yh += theta[1 + k] * F[i * K + k];
    const double e = y[i] - yh, c = y[i] - ybar;
    ssr += e * e;
    sst += c * c;
  }
  ssr = wave_sum(ssr);
  sst = wave_sum(sst);
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = ssr;
    red[1][tid >> 6] = sst;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < FIT_THREADS / 64; ++w) {
      a += red[0][w];
      b += red[1][w];
    }
    acc[FA_SSR] += a;
    acc[FA_SST] += b;
  }
}

__global__ void k_fit_r2(const double* acc, double* r2) {
  if (threadIdx.x == 0) r2[0] = 1.0 - acc[FA_SSR] / acc[FA_SST];
}

// Regression over n fields s [n][L][N] with targets y [n], in chunks of up to
// max_batch fields whose features go to the plan's F_old buffer.
int launch_fit_chunked(Plan& p, const Eff& e, long n, const int8_t* s, const double* y, double* theta, double* r2,
                       hipStream_t st) {
  const long per = (long)p.L * p.n, C = p.max_batch;
  const int K = e.n_terms;
  for (long c0 = 0; c0 < n; c0 += C) {
    const long rows = std::min(C, n - c0);
    SLQ_TRY(launch_features(p, e, rows, s + c0 * per, p.F_old, st));
    k_fit_acc<<<1, FIT_THREADS, 0, st>>>(c0 == 0, rows, K, p.F_old, y + c0, p.fit_acc);
    SLQ_LAUNCHED();
  }
  k_fit_solve<<<1, FIT_THREADS, 0, st>>>(K, p.fit_acc, theta);
  SLQ_LAUNCHED();
  for (long c0 = 0; c0 < n; c0 += C) {
    const long rows = std::min(C, n - c0);
    SLQ_TRY(launch_features(p, e, rows, s + c0 * per, p.F_old, st));
    k_fit_resid<<<1, FIT_THREADS, 0, st>>>(rows, K, p.F_old, y + c0, theta, p.fit_acc);
    SLQ_LAUNCHED();
  }
  k_fit_r2<<<1, 64, 0, st>>>(p.fit_acc, r2);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

static int efail(int code, const char* msg) {
  set_error(msg);
  return code;
}

// Byte layout of an effective model's device tables for N sites and n_terms
// terms (sizes bounded without the colouring: at most N colours, 25 spatial
// offsets, two partner relations per offset and term), including the copy of
// the network's parameters and the move colouring used while one is attached.
struct EffLayout {
  size_t terms, theta, sites, off, shoff, shd, pairs, uoff, net, nsites, noff, total;
};
static EffLayout eff_layout(int N, int n_terms) {
  EffLayout l{};
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t r = o;
    o += (b + 255) / 256 * 256;
    return r;
  };
  l.terms = take(8 * (size_t)n_terms);
  l.theta = take(8 * (size_t)(1 + n_terms));
  l.sites = take(4 * (size_t)N);
  l.off = take(4 * (size_t)(N + 1));
  l.shoff = take(4 * (size_t)(MAX_SHELL + 2));
  l.shd = take(4 * 50);
  l.pairs = take(4 * (size_t)n_terms * 50);
  l.uoff = take(4 * 50);
  l.net = take(8 * (size_t)SLQ_NET_PARAMS);
  l.nsites = take(4 * (size_t)N);
  l.noff = take(4 * (size_t)(N + 1));
  l.total = o;
  return l;
}

}  // namespace slq

using namespace slq;

extern "C" {

int slq_eff_workspace_size(const slq_plan* plan, int32_t n_terms, size_t* bytes) {
  if (!plan || !bytes) return efail(SLQ_ERR_ARG, "NULL argument");
  if (n_terms < 1 || n_terms > MAX_TERMS) return efail(SLQ_ERR_ARG, "n_terms must be in [1, 64]");
  *bytes = eff_layout(plan->p.n, n_terms).total;
  return SLQ_OK;
}

int slq_eff_create(slq_plan* plan, int32_t n_terms, const int32_t* terms, const double* lambda, double c0,
                   void* d_work, size_t work_bytes, slq_eff** out) {
  if (!plan || !out || !terms || !lambda) return efail(SLQ_ERR_ARG, "NULL argument");
  *out = nullptr;
  Plan& p = plan->p;
  if (n_terms < 1 || n_terms > MAX_TERMS) return efail(SLQ_ERR_ARG, "n_terms must be in [1, 64]");
  const int lx = p.m.lx, ly = p.m.ly, N = p.n, L = p.L;
  std::vector<std::set<int>> nbr(N);
  for (int k = 0; k < n_terms; ++k) {
    const int r = terms[2 * k], dl = terms[2 * k + 1];
    if (r < 0 || r > MAX_SHELL || dl < 0 || dl > L / 2) return efail(SLQ_ERR_ARG, "unusable term (r, dl)");
    if (r == 0 && dl == 0) continue;  // one-body term: no partners
    if (dl == 0) {
      for (int o = kShellOff[r]; o < kShellOff[r + 1]; ++o) {
        const int dx = ((kShellDxy[o][0] % lx) + lx) % lx, dy = ((kShellDxy[o][1] % ly) + ly) % ly;
        if (dx == 0 && dy == 0) return efail(SLQ_ERR_ARG, "a term makes a site its own partner on this lattice");
      }
      for (int i = 0; i < N; ++i) {
        const int x = i % lx, y = i / lx;
        for (int o = kShellOff[r]; o < kShellOff[r + 1]; ++o) {
          const int j = ((x + kShellDxy[o][0]) % lx + lx) % lx + lx * (((y + kShellDxy[o][1]) % ly + ly) % ly);
          if (j != i) {
            nbr[i].insert(j);
            nbr[j].insert(i);
          }
        }
      }
    }
  }
  // greedy colouring, ascending site index, smallest free colour
  std::vector<int> col(N, -1);
  int nc = 0;
  for (int i = 0; i < N; ++i) {
    std::set<int> used;
    for (int j : nbr[i])
      if (col[j] >= 0) used.insert(col[j]);
    int c = 0;
    while (used.count(c)) ++c;
    col[i] = c;
    nc = std::max(nc, c + 1);
  }
  std::vector<int32_t> sites, off(nc + 1, 0);
  int maxc = 0;
  for (int c = 0; c < nc; ++c) {
    off[c] = (int32_t)sites.size();
    for (int i = 0; i < N; ++i)
      if (col[i] == c) sites.push_back(i);
    maxc = std::max(maxc, (int)sites.size() - off[c]);
  }
  off[nc] = (int32_t)sites.size();
  std::vector<int32_t> pairs, uoff;
  int uidx[25];
  for (int o = 0; o < 25; ++o) uidx[o] = -1;
  for (int k = 0; k < n_terms; ++k) {
    const int r = terms[2 * k], dl = terms[2 * k + 1];
    if (r == 0 && dl == 0) continue;
    for (int o = kShellOff[r]; o < kShellOff[r + 1]; ++o) {
      if (uidx[o] < 0) {
        uidx[o] = (int)uoff.size() / 2;
        uoff.push_back(kShellDxy[o][0]);
        uoff.push_back(kShellDxy[o][1]);
      }
      for (int sg = (dl == 0 ? 0 : -1); sg <= (dl == 0 ? 0 : 1); sg += 2) {
        const int dt = sg * dl;
        pairs.push_back(uidx[o] | ((dt + 2048) << 8) | (k << 20));
      }
    }
  }
  std::vector<double> theta(1 + n_terms);
  theta[0] = c0;
  for (int k = 0; k < n_terms; ++k) theta[1 + k] = lambda[k];
  std::vector<int32_t> shoff(kShellOff, kShellOff + MAX_SHELL + 2);
  std::vector<int32_t> shd(2 * 25);
  for (int o = 0; o < 25; ++o) {
    shd[2 * o] = kShellDxy[o][0];
    shd[2 * o + 1] = kShellDxy[o][1];
  }
  slq_eff* h = new (std::nothrow) slq_eff();
  if (!h) return efail(SLQ_ERR_DEVICE, "host allocation failed");
  Eff& e = h->e;
  e.plan = &p;
  e.n_terms = n_terms;
  e.h_terms.assign(terms, terms + 2 * n_terms);
  e.n_colours = nc;
  e.n_classes = nc * L;
  e.max_class = maxc;
  const size_t b_terms = 8 * n_terms, b_theta = 8 * (1 + n_terms), b_sites = 4 * N, b_off = 4 * (nc + 1),
               b_shoff = 4 * shoff.size(), b_shd = 4 * shd.size();
  const EffLayout lay = eff_layout(N, n_terms);
  if (d_work && work_bytes < lay.total) {
    delete h;
    return efail(SLQ_ERR_WORKSPACE, "eff workspace smaller than slq_eff_workspace_size");
  }
  if (d_work && ((uintptr_t)d_work & 255)) {
    delete h;
    return efail(SLQ_ERR_ARG, "d_work must be 256-byte aligned");
  }
  char* base = (char*)d_work;
  if (hipSetDevice(p.device) != hipSuccess || (!base && hipMalloc((void**)&base, lay.total) != hipSuccess)) {
    delete h;
    return efail(SLQ_ERR_DEVICE, "hipMalloc failed");
  }
  e.base = base;
  e.owns_base = d_work == nullptr;
  const size_t o1 = lay.terms, o2 = lay.theta, o3 = lay.sites, o4 = lay.off, o5 = lay.shoff, o6 = lay.shd,
               o7 = lay.pairs, o8 = lay.uoff;
  e.d_net = (double*)(base + lay.net);
  e.d_ncol_sites = (int32_t*)(base + lay.nsites);
  e.d_ncol_off = (int32_t*)(base + lay.noff);
  e.d_terms = (int32_t*)(base + o1);
  e.d_theta = (double*)(base + o2);
  e.d_col_sites = (int32_t*)(base + o3);
  e.d_col_off = (int32_t*)(base + o4);
  e.d_shell_off = (int32_t*)(base + o5);
  e.d_shell_dxy = (int32_t*)(base + o6);
  e.d_pairs = (int32_t*)(base + o7);
  e.n_pairs = (int)pairs.size();
  e.d_uoff = (int32_t*)(base + o8);
  e.n_uoff = (int)uoff.size() / 2;
  bool ok = (pairs.empty() ||
             hipMemcpy(e.d_pairs, pairs.data(), 4 * pairs.size(), hipMemcpyHostToDevice) == hipSuccess) &&
            (uoff.empty() || hipMemcpy(e.d_uoff, uoff.data(), 4 * uoff.size(), hipMemcpyHostToDevice) == hipSuccess) &&
            hipMemcpy(e.d_terms, terms, b_terms, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(e.d_theta, theta.data(), b_theta, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(e.d_col_sites, sites.data(), b_sites, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(e.d_col_off, off.data(), b_off, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(e.d_shell_off, shoff.data(), b_shoff, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(e.d_shell_dxy, shd.data(), b_shd, hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    if (e.owns_base) hipFree(base);
    delete h;
    return efail(SLQ_ERR_DEVICE, "hipMemcpy failed");
  }
  *out = h;
  return SLQ_OK;
}

int slq_eff_destroy(slq_eff* eff) {
  if (!eff) return SLQ_OK;
  hipSetDevice(eff->e.plan->device);
  hipDeviceSynchronize();
  if (eff->e.owns_base) hipFree(eff->e.base);
  delete eff;
  return SLQ_OK;
}

int slq_eff_set_net(slq_eff* eff, const double* d_params, int32_t net_prec, hipStream_t stream) {
  if (!eff) return efail(SLQ_ERR_ARG, "eff is NULL");
  Eff& e = eff->e;
  Plan& p = *e.plan;
  if (!d_params) {
    e.net_on = false;
    return SLQ_OK;
  }
  // Proposals need a move kernel that is reversible with respect to the
  // action Eq. 4 charges.  The move kernel updates the network's activations
  // incrementally on every accepted flip; in FP32 those updates round
  // differently along different paths, so a move and its reverse would not
  // change the action by exact negatives.  FP64 keeps that to round-off.
  if (net_prec != SLQ_PREC_FP64)
    return efail(SLQ_ERR_ARG, "net_prec must be SLQ_PREC_FP64 for proposals (FP32 is for training and forward passes)");
  if (p.m.lx < 5 || p.m.ly < 5 || p.L < 5)
    return efail(SLQ_ERR_ARG, "moves with the learned action need lx, ly and L >= 5");
  SLQ_HIP(hipSetDevice(p.device));
  if (e.n_ncolours == 0) {  // first attach: the colouring that separates the network's reach
    // colouring of the graph of dl = 0 couplings plus spatial Chebyshev distance <= 4
    const int lx = p.m.lx, ly = p.m.ly, N = p.n;
    std::vector<std::set<int>> nbr(N);
    for (int k = 0; k < e.n_terms; ++k) {
      const int r = e.h_terms[2 * k], dl = e.h_terms[2 * k + 1];
      if (dl != 0) continue;
      for (int i = 0; i < N; ++i) {
        const int x = i % lx, y = i / lx;
        for (int o = kShellOff[r]; o < kShellOff[r + 1]; ++o) {
          const int j = ((x + kShellDxy[o][0]) % lx + lx) % lx + lx * (((y + kShellDxy[o][1]) % ly + ly) % ly);
          if (j != i) nbr[i].insert(j);
        }
      }
    }
    for (int i = 0; i < N; ++i) {
      const int x = i % lx, y = i / lx;
      for (int dy = -4; dy <= 4; ++dy)
        for (int dx = -4; dx <= 4; ++dx) {
          const int j = ((x + dx) % lx + lx) % lx + lx * (((y + dy) % ly + ly) % ly);
          if (j != i) nbr[i].insert(j);
        }
    }
    std::vector<int> col(N, -1);
    int nc = 0;
    for (int i = 0; i < N; ++i) {
      std::set<int> used;
      for (int j : nbr[i])
        if (col[j] >= 0) used.insert(col[j]);
      int c = 0;
      while (used.count(c)) ++c;
      col[i] = c;
      nc = std::max(nc, c + 1);
    }
    std::vector<int32_t> sites, off(nc + 1, 0);
    for (int c = 0; c < nc; ++c) {
      off[c] = (int32_t)sites.size();
      for (int i = 0; i < N; ++i)
        if (col[i] == c) sites.push_back(i);
    }
    off[nc] = (int32_t)sites.size();
    const size_t b_sites = 4 * N, b_off = 4 * (nc + 1);
    if (hipMemcpy(e.d_ncol_sites, sites.data(), b_sites, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(e.d_ncol_off, off.data(), b_off, hipMemcpyHostToDevice) != hipSuccess)
      return efail(SLQ_ERR_DEVICE, "hipMemcpy failed");
    e.n_ncolours = nc;
  }
  int rc = copy_f64(d_params, e.d_net, SLQ_NET_PARAMS, stream);
  if (rc != SLQ_OK) return rc;
  e.net_prec = net_prec;
  e.net_on = true;
  return SLQ_OK;
}

int slq_eff_net_classes(const slq_eff* eff, int32_t* n_classes) {
  if (!eff || !n_classes) return efail(SLQ_ERR_ARG, "NULL argument");
  if (eff->e.n_ncolours == 0) return efail(SLQ_ERR_ARG, "no network attached");
  *n_classes = eff->e.n_ncolours * eff->e.plan->L;
  return SLQ_OK;
}

int slq_eff_classes(const slq_eff* eff, int32_t* n_classes) {
  if (!eff || !n_classes) return efail(SLQ_ERR_ARG, "NULL argument");
  *n_classes = eff->e.n_classes;
  return SLQ_OK;
}

int slq_eff_set_theta(slq_eff* eff, const double* d_theta, hipStream_t stream) {
  if (!eff || !d_theta) return efail(SLQ_ERR_ARG, "NULL argument");
  SLQ_HIP(hipSetDevice(eff->e.plan->device));
  return copy_f64(d_theta, eff->e.d_theta, 1 + eff->e.n_terms, stream);
}

int slq_eff_sweep(slq_plan* plan, const slq_eff* eff, int32_t batch, int8_t* d_s, int32_t n_moves, uint64_t seed,
                  uint64_t step, uint64_t chain0, int64_t* d_accepts, double* d_dS, hipStream_t stream) {
  if (!plan || !eff || !d_s) return efail(SLQ_ERR_ARG, "NULL argument");
  Plan& p = plan->p;
  if (eff->e.plan != &p) return efail(SLQ_ERR_ARG, "eff belongs to another plan");
  if (batch < 0 || n_moves < 0) return efail(SLQ_ERR_ARG, "batch and n_moves must be >= 0");
  SLQ_HIP(hipSetDevice(p.device));
  return launch_eff_sweep(p, eff->e, batch, d_s, n_moves, seed, step, chain0, d_accepts, d_dS, stream);
}

int slq_eff_features(slq_plan* plan, const slq_eff* eff, int32_t batch, const int8_t* d_s, double* d_F,
                     hipStream_t stream) {
  if (!plan || !eff || !d_s || !d_F) return efail(SLQ_ERR_ARG, "NULL argument");
  if (eff->e.plan != &plan->p) return efail(SLQ_ERR_ARG, "eff belongs to another plan");
  if (batch < 0) return efail(SLQ_ERR_ARG, "batch must be >= 0");
  SLQ_HIP(hipSetDevice(plan->p.device));
  return launch_features(plan->p, eff->e, batch, d_s, d_F, stream);
}

int slq_cumulative_step(slq_plan* plan, const slq_eff* eff, int32_t batch, int8_t* d_s, double* d_logabs,
                        int8_t* d_sign, int32_t n_moves, uint64_t seed, uint64_t step, uint64_t chain0,
                        int8_t* d_accepted, double* d_logA, int32_t* d_status, hipStream_t stream) {
  if (!plan || !eff || !d_s || !d_logabs || !d_sign) return efail(SLQ_ERR_ARG, "NULL argument");
  Plan& p = plan->p;
  const Eff& e = eff->e;
  if (e.plan != &p) return efail(SLQ_ERR_ARG, "eff belongs to another plan");
  int rc = check_batch(p, batch);
  if (rc != SLQ_OK) return rc;
  if (batch == 0) return SLQ_OK;
  if (n_moves < 0) return efail(SLQ_ERR_ARG, "n_moves must be >= 0");
  SLQ_HIP(hipSetDevice(p.device));
  const long per = (long)p.L * p.n;
  int32_t* status = d_status ? d_status : p.status;
  if ((rc = fill_i32(status, batch, 0, stream)) != SLQ_OK) return rc;
  if ((rc = copy_i8(d_s, p.s_work, per * batch, stream)) != SLQ_OK) return rc;
  if ((rc = launch_eff_sweep(p, e, batch, p.s_work, n_moves, seed, step, chain0, nullptr, nullptr, stream)) != SLQ_OK)
    return rc;
  if ((rc = launch_features(p, e, batch, d_s, p.F_old, stream)) != SLQ_OK) return rc;
  if ((rc = launch_features(p, e, batch, p.s_work, p.F_new, stream)) != SLQ_OK) return rc;
  if ((rc = launch_check_spins(p, batch, d_s, status, stream)) != SLQ_OK) return rc;
  double *sn_old = nullptr, *sn_new = nullptr;
  if (e.net_on && (rc = net_pair(p, e, batch, d_s, p.s_work, &sn_old, &sn_new, stream)) != SLQ_OK) return rc;
  rc = run_chain(p, batch, p.s_work, 0, status, stream);
  if (rc == SLQ_OK) rc = launch_finish(p, batch, nullptr, p.dvec, p.sgn_work, status, stream);
  if (rc != SLQ_OK) return rc;
  return launch_accept(p, e, batch, d_s, p.s_work, d_logabs, d_sign, p.dvec, p.sgn_work, p.F_old, p.F_new, sn_old,
                       sn_new, seed, step, chain0, d_accepted, d_logA, stream);
}

int slq_fit_effective(slq_plan* plan, const slq_eff* eff, int64_t n_samples, const int8_t* d_S,
                      const double* d_logabs, double* d_theta, double* d_r2, hipStream_t stream) {
  if (!plan || !eff || !d_S || !d_logabs || !d_theta || !d_r2) return efail(SLQ_ERR_ARG, "NULL argument");
  Plan& p = plan->p;
  const Eff& e = eff->e;
  if (e.plan != &p) return efail(SLQ_ERR_ARG, "eff belongs to another plan");
  if (n_samples < e.n_terms + 2) return efail(SLQ_ERR_ARG, "n_samples must be >= n_terms + 2");
  SLQ_HIP(hipSetDevice(p.device));
  return launch_fit_chunked(p, e, n_samples, d_S, d_logabs, d_theta, d_r2, stream);
}

}  // extern "C"
