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
  const size_t lds = sizeof(double) * ((size_t)p.n + SWEEP_KD + 4);
  allow_max_lds((const void*)k_flip_slice);
  k_flip_slice<<<batch, FL_THREADS, lds, st>>>(f);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

// drift[b] = max(drift[b], max |Gw - Gf|); Gw <- Gf
__global__ __launch_bounds__(256) void k_drift_replace(int N, double* __restrict__ Gw, const double* __restrict__ Gf,
                                                       double* drift) {
  __shared__ double red[4];
  const int b = blockIdx.x;
  const long NN = (long)N * N;
  double m = 0.0;
  for (long idx = threadIdx.x; idx < NN; idx += 256) {
    const double f = Gf[b * NN + idx];
    const double d = fabs(Gw[b * NN + idx] - f);
    m = (d > m || d != d) ? d : m;
    Gw[b * NN + idx] = f;
  }
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    drift[b] = fmax(drift[b], t);
  }
}

int launch_drift(Plan& p, int batch, double* Gw, const double* Gf, double* drift, hipStream_t st) {
  k_drift_replace<<<batch, 256, 0, st>>>(p.n, Gw, Gf, drift);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

}  // namespace slq
