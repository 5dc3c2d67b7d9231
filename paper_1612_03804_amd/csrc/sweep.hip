// Local-update DQMC sweep ("Basics of DQMC"): O(1) determinant ratio per
// proposed flip and O(N^2) Green's-function update per accepted flip.
//
// Flipping s_{i,l} multiplies B_l on the right by 1 + delta e_i e_i^T with
// delta = exp(2 dtau xi s_{i,l}) - 1.  With G the Green's function of the
// cyclic chain whose rightmost factor is B_l,
//     R = 1 + delta (1 - G_ii),
// accepted iff u < |R|, and then (Sherman-Morrison)
//     G <- G - a x y^T,  a = delta / R,  x = e_i - G[:, i],  y = G[i, :].
// Updates are delayed: up to KD accepted flips are kept as (a_m, x_m, y_m)
// and the current column, row and diagonal of G are formed from
// G_0 - sum_m a_m x_m y_m^T on demand; the rank-KD correction is applied to
// G_0 when the buffer fills and at the end of the slice.  The diagonal of the
// current G is carried in LDS so the ratio of every proposal costs O(1).
#include "slq_internal.h"

namespace slq {

constexpr int FL_THREADS = 512;
constexpr int FL_WAVES = FL_THREADS / 64;

struct FlipArgs {
  int N, L;
  int8_t* s;          // [batch][L][N]
  double* G;          // [batch][N][N]
  double* logabs;     // [batch]
  int8_t* sign;       // [batch]
  int64_t* accepts;   // [batch]
  double* X;          // [batch][N][KD]
  double* Y;          // [batch][KD][N]
  int slice;          // 0-based slice l-1
  double a;           // dtau * xi
  uint64_t seed, sweep, chain0;
};

__device__ void flush_rank(double* __restrict__ G, const double* __restrict__ X, const double* __restrict__ Y,
                           const double* A, int N, int k) {
  const long NN = (long)N * N;
  for (long idx = threadIdx.x; idx < NN; idx += FL_THREADS) {
    const int r = (int)(idx / N), c = (int)(idx % N);
    double s = 0.0;
    for (int m = 0; m < k; ++m) s += A[m] * X[(long)r * SWEEP_KD + m] * Y[(long)m * N + c];
    G[idx] -= s;
  }
}

__global__ __launch_bounds__(FL_THREADS) void k_flip_slice(FlipArgs f) {
  extern __shared__ double lds[];
  const int N = f.N;
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const long NN = (long)N * N;
  double* G = f.G + b * NN;
  int8_t* s = f.s + (long)b * f.L * N + (long)f.slice * N;
  double* X = f.X + (long)b * N * SWEEP_KD;
  double* Y = f.Y + (long)b * SWEEP_KD * N;
  double* diag = lds;               // [N] diagonal of the current G
  double* A = diag + N;             // [KD]
  double* shared2 = A + SWEEP_KD;   // [2][2]: accept flag and a = delta/R, by site parity

  for (int r = tid; r < N; r += FL_THREADS) diag[r] = G[(long)r * N + r];
  __syncthreads();

  const uint64_t chain = f.chain0 + b;
  double la = 0.0;
  int neg = 0;
  int64_t nacc = 0;
  int k = 0;
  for (int i = 0; i < N; ++i) {
    // the decision of site i is broadcast through a slot that alternates with
    // i, so thread 0 can publish site i+1 while slower waves still read site i
    double* shared = shared2 + 2 * (i & 1);
    if (tid == 0) {
      const double si = (double)s[i];
      const double delta = exp(2.0 * f.a * si) - 1.0;
      const double R = 1.0 + delta * (1.0 - diag[i]);
      const double u = philox_uniform((uint64_t)i, (uint64_t)f.slice, f.sweep, chain, f.seed, TAG_LOCAL);
      const bool acc = u < fabs(R);
      shared[0] = acc ? 1.0 : 0.0;
      shared[1] = delta / R;
      if (acc) {
        s[i] = (int8_t)(-s[i]);
        la += log(fabs(R));
        neg ^= (R < 0.0);
        ++nacc;
      }
    }
    __syncthreads();
    if (shared[0] != 0.0) {
      const double a = shared[1];
      // current column x = e_i - G[:, i] and row y = G[i, :]
      for (int r = tid; r < N; r += FL_THREADS) {
        double gc = G[(long)r * N + i];
        double gr = G[(long)i * N + r];
        for (int m = 0; m < k; ++m) {
          gc -= A[m] * X[(long)r * SWEEP_KD + m] * Y[(long)m * N + i];
          gr -= A[m] * X[(long)i * SWEEP_KD + m] * Y[(long)m * N + r];
        }
        const double x = (r == i ? 1.0 : 0.0) - gc;
        X[(long)r * SWEEP_KD + k] = x;
        Y[(long)k * N + r] = gr;
      }
      __syncthreads();
      for (int r = tid; r < N; r += FL_THREADS) diag[r] -= a * X[(long)r * SWEEP_KD + k] * Y[(long)k * N + r];
      if (tid == 0) A[k] = a;
      ++k;
      __syncthreads();
      if (k == SWEEP_KD) {
        flush_rank(G, X, Y, A, N, k);
        k = 0;
        __syncthreads();
      }
    }
  }
  if (k > 0) flush_rank(G, X, Y, A, N, k);
  if (tid == 0) {
    f.logabs[b] += la;
    if (neg) f.sign[b] = (int8_t)(-f.sign[b]);
    f.accepts[b] += nacc;
  }
}

// The same sweep for N <= FF_MAXN with the delayed-update factors on chip:
// thread c owns column c, keeps y_m[c] (m < KD) in registers and writes x_m[c]
// into an LDS table X[c][m].  For site i every thread forms its entry of the
// current column and row of G,
//     G[c][i] = G_0[c][i] - sum_m a_m x_m[c] y_m[i],   G[i][c] = G_0[i][c] - sum_m a_m x_m[i] y_m[c],
// from G_0 values fetched FF_PD sites ahead, the y_m[i] published by thread i
// and the x_m[i] read from the table; the rank-KD flush runs on the matrix
// cores from the same table.  The spins, the uniforms and
// the two possible deltas of the slice are prepared in LDS first, so the
// decision of a site reads LDS only.  One barrier per rejected site, two per
// accepted site; these order LDS traffic only, so the fetches of G_0 stay in
// flight across them.
// KD: depth of the delayed update (flushes per slice N / KD, each reading and
// writing G): 20 where the LDS holds its tables, else 16.
constexpr int FF_MAXN = FL_THREADS, FF_PD = 4;

typedef double fd4_t __attribute__((ext_vector_type(4)));

// G_0 -= X diag(a) Y on the matrix cores: X [N][k] is the LDS table, AY [k][N]
// holds a_m y_m (written by the column owners), unused slots are zero.  Wave w
// takes the 16 x 16 tiles w, w + 8, ...; a tile of G_0 is fetched one tile
// ahead.  Lane l holds rows l/16 + 4q and column l%16 of its tile, the
// operand and result layout of v_mfma_f64_16x16x4_f64.
template <int KD>
__device__ __forceinline__ void flush_mfma(double* __restrict__ G, int N, const double* __restrict__ Xs,
                                           const double* __restrict__ AY, int ldy) {
  constexpr int XP = KD + 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nt = (N + 15) / 16, tiles = nt * nt;
  auto load = [&](int t, fd4_t& v) {
    const int tr = t / nt, tc = t % nt, col = tc * 16 + (lane & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = tr * 16 + (lane >> 4) + 4 * q;
      v[q] = (t < tiles && row < N && col < N) ? G[(long)row * N + col] : 0.0;
    }
  };
  fd4_t cur, nxt;
  load(wave, cur);
  for (int t = wave; t < tiles; t += FL_WAVES) {
    load(t + FL_WAVES, nxt);
    const int tr = t / nt, tc = t % nt, col = tc * 16 + (lane & 15), xrow = tr * 16 + (lane & 15);
#pragma unroll
    for (int ks = 0; ks < KD; ks += 4) {
      const int kk = ks + (lane >> 4);
      const double xa = xrow < N ? -Xs[(long)xrow * XP + kk] : 0.0;
      const double yb = col < N ? AY[(long)kk * ldy + col] : 0.0;
      cur = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, yb, cur, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = tr * 16 + (lane >> 4) + 4 * q;
      if (row < N && col < N) G[(long)row * N + col] = cur[q];
    }
    cur = nxt;
  }
}

template <int KD>
__global__ __launch_bounds__(FL_THREADS) void k_flip_fast(FlipArgs f) {
  static_assert(KD % 4 == 0, "the flush takes KD in steps of 4");
  constexpr int FF_KD = KD, FF_XP = KD + 2;
  extern __shared__ double lds[];
  const int N = f.N;
  const int b = blockIdx.x;
  const int c = threadIdx.x;
  const bool own = c < N;
  const long NN = (long)N * N;
  double* G = f.G + b * NN;
  int8_t* s = f.s + (long)b * f.L * N + (long)f.slice * N;
  double* Xs = lds;                     // [N][FF_XP] x_m[r] at Xs[r * FF_XP + m]
  double* diag = Xs + (long)N * FF_XP;  // [N] diagonal of the current G
  double* U = diag + N;                 // [N] uniform of each site
  double* A = U + N;                    // [KD] a_m
  double* yi = A + FF_KD;               // [KD] y_m[i] of the current site
  double* shared2 = yi + FF_KD;         // [2][2] decision of the site, by parity
  const int ldy = N + 1;
  double* AY = shared2 + 4;             // [KD][N + 1] a_m y_m[c] for the flush
  int* sp = (int*)(AY + (long)FF_KD * ldy);  // [N] spins of the slice

  const uint64_t chain = f.chain0 + b;
  for (int q = c; q < N * FF_XP; q += FL_THREADS) Xs[q] = 0.0;  // unused slots enter the flush times zero
  if (own) {
    diag[c] = G[(long)c * N + c];
    sp[c] = s[c];
    U[c] = philox_uniform((uint64_t)c, (uint64_t)f.slice, f.sweep, chain, f.seed, TAG_LOCAL);
  }
  const double dplus = exp(2.0 * f.a) - 1.0, dminus = exp(-2.0 * f.a) - 1.0;  // delta for s = +1, -1
  double y[FF_KD];
#pragma unroll
  for (int m = 0; m < FF_KD; ++m) y[m] = 0.0;
  // G_0[c][i] and G_0[i][c] for the sites of the current and of the next group of FF_PD
  double pc[FF_PD], pr[FF_PD], nc[FF_PD], nr[FF_PD];
  auto fetch = [&](double(&col)[FF_PD], double(&row)[FF_PD], int i0) {
#pragma unroll
    for (int j = 0; j < FF_PD; ++j) {
      const int i = i0 + j;
      col[j] = (own && i < N) ? G[(long)c * N + i] : 0.0;
      row[j] = (own && i < N) ? G[(long)i * N + c] : 0.0;
    }
  };
  fetch(pc, pr, 0);
  fetch(nc, nr, FF_PD);
  lds_barrier();

  double la = 0.0;
  int neg = 0;
  int64_t nacc = 0;
  int k = 0;
  for (int i0 = 0; i0 < N; i0 += FF_PD) {
#pragma unroll
    for (int j = 0; j < FF_PD; ++j) {
      const int i = i0 + j;
      if (i >= N) break;  // uniform
      double* shared = shared2 + 2 * (i & 1);
      if (c == 0) {
        const int si = sp[i];
        const double delta = si > 0 ? dplus : dminus;
        const double R = 1.0 + delta * (1.0 - diag[i]);
        const bool acc = U[i] < fabs(R);
        shared[0] = acc ? 1.0 : 0.0;
        shared[1] = delta / R;
        if (acc) {
          sp[i] = -si;
          la += log(fabs(R));
          neg ^= (R < 0.0);
          ++nacc;
        }
      }
      if (c == i) {
#pragma unroll
        for (int m = 0; m < FF_KD; ++m)
          if (m < k) yi[m] = y[m];
      }
      lds_barrier();
      if (shared[0] == 0.0) continue;  // uniform
      const double a = shared[1];
      if (own) {
        double gc = pc[j], gr = pr[j];
        const double* xr = Xs + (long)c * FF_XP;
        const double* xi = Xs + (long)i * FF_XP;
#pragma unroll
        for (int m = 0; m < FF_KD; ++m)
          if (m < k) {
            gc -= A[m] * xr[m] * yi[m];
            gr -= A[m] * xi[m] * y[m];
          }
        const double x = (c == i ? 1.0 : 0.0) - gc;
        Xs[(long)c * FF_XP + k] = x;
#pragma unroll
        for (int m = 0; m < FF_KD; ++m)
          if (m == k) y[m] = gr;
        diag[c] -= a * x * gr;
      }
      if (c == 0) A[k] = a;
      ++k;
      lds_barrier();
      if (k == FF_KD) {  // G_0 -= sum_m a_m x_m y_m^T
        if (own) {
#pragma unroll
          for (int m = 0; m < FF_KD; ++m) {
            AY[(long)m * ldy + c] = A[m] * y[m];
            y[m] = 0.0;
          }
        }
        lds_barrier();
        flush_mfma<KD>(G, N, Xs, AY, ldy);
        k = 0;
        __syncthreads();
        // the fetched G_0 values predate the flush: fetch the rest of this group and the next again
#pragma unroll
        for (int j2 = 0; j2 < FF_PD; ++j2) {
          const int i2 = i0 + j2;
          if (j2 > j) {
            pc[j2] = (own && i2 < N) ? G[(long)c * N + i2] : 0.0;
            pr[j2] = (own && i2 < N) ? G[(long)i2 * N + c] : 0.0;
          }
        }
        fetch(nc, nr, i0 + FF_PD);
      }
    }
#pragma unroll
    for (int j = 0; j < FF_PD; ++j) {
      pc[j] = nc[j];
      pr[j] = nr[j];
    }
    fetch(nc, nr, i0 + 2 * FF_PD);
  }
  if (k > 0) {
    if (own) {
#pragma unroll
      for (int m = 0; m < FF_KD; ++m) AY[(long)m * ldy + c] = m < k ? A[m] * y[m] : 0.0;
    }
    lds_barrier();
    flush_mfma<KD>(G, N, Xs, AY, ldy);
  }
  __syncthreads();  // the decisions of every site are in sp
  if (own) s[c] = (int8_t)sp[c];
  if (c == 0) {
    f.logabs[b] += la;
    if (neg) f.sign[b] = (int8_t)(-f.sign[b]);
    f.accepts[b] += nacc;
  }
}

int launch_flip_slice(Plan& p, int batch, int8_t* s, double* G, double* logabs, int8_t* sign, int slice,
                      uint64_t seed, uint64_t sweep, uint64_t chain0, int64_t* accepts, hipStream_t st) {
  FlipArgs f;
  f.N = p.n;
  f.L = p.L;
  f.s = s;
  f.G = G;
  f.logabs = logabs;
  f.sign = sign;
  f.accepts = accepts;
  f.X = p.dX;
  f.Y = p.dY;
  f.slice = slice;
  f.a = p.m.dtau * p.m.xi;
  f.seed = seed;
  f.sweep = sweep;
  f.chain0 = chain0;
  if (p.n <= FF_MAXN) {
    auto lds_of = [&](size_t kd) {
      return sizeof(double) * ((size_t)p.n * (kd + 2) + 2 * p.n + 2 * kd + 4 + kd * (p.n + 1)) + sizeof(int) * p.n;
    };
    if (lds_of(20) <= 160 * 1024) {
      allow_max_lds((const void*)k_flip_fast<20>);
      k_flip_fast<20><<<batch, FL_THREADS, lds_of(20), st>>>(f);
    } else {
      allow_max_lds((const void*)k_flip_fast<16>);
      k_flip_fast<16><<<batch, FL_THREADS, lds_of(16), st>>>(f);
    }
    SLQ_LAUNCHED();
    return SLQ_OK;
  }
  const size_t lds = sizeof(double) * ((size_t)p.n + SWEEP_KD + 4);
  allow_max_lds((const void*)k_flip_slice);
  k_flip_slice<<<batch, FL_THREADS, lds, st>>>(f);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

// drift[b] = max(drift[b], max |Gw - Gf|); Gw <- Gf.  The maximum propagates
// NaN (a non-finite wrapped G must show in the drift), and a non-finite drift
// sets SLQ_ST_NONFINITE in status[b].
__global__ __launch_bounds__(256) void k_drift_replace(int N, double* __restrict__ Gw, const double* __restrict__ Gf,
                                                       double* drift, int32_t* status) {
  __shared__ double red[4];
  const int b = blockIdx.x;
  const long NN = (long)N * N;
  double m = 0.0;
  for (long idx = threadIdx.x; idx < NN; idx += 256) {
    const double f = Gf[b * NN + idx];
    const double d = fabs(Gw[b * NN + idx] - f);
    m = nan_max(m, d);
    Gw[b * NN + idx] = f;
  }
  m = wave_max_nan(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = nan_max(nan_max(red[0], red[1]), nan_max(red[2], red[3]));
    const double d = nan_max(drift[b], t);
    drift[b] = d;
    if (!isfinite(d) && status) status[b] |= SLQ_ST_NONFINITE;
  }
}

int launch_drift(Plan& p, int batch, double* Gw, const double* Gf, double* drift, int32_t* status, hipStream_t st) {
  k_drift_replace<<<batch, 256, 0, st>>>(p.n, Gw, Gf, drift, status);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

}  // namespace slq
