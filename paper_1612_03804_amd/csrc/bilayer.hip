// The paper's own workload ("Results", Eq. 6): four fermion flavours on a
// bilayer coupled to transverse-field Ising spins.  Flavour (lambda, sigma)
// sees the potential -xi s eta with eta = sigma in layer 1 and -sigma in
// layer 2; with no interlayer hopping the flavours do not mix, and in the
// single-flavour form of the hot path (d_l = exp(-dtau xi s)) two flavours
// give W_f(s) and two W_f(-s):
//     omega(s) = phi(s) [W_f(s) W_f(-s)]^2  (sign-free),
//     ln phi  = dtau J sum_l sum_<ij> s_{i,l} s_{j,l} + K_tau sum_{i,l} s_{i,l} s_{i,l+1},
//     K_tau   = -1/2 ln tanh(dtau h),
// phi being the weight of the Ising spins alone (Eq. 1's fermion-free factor; the
// quantum-to-classical mapping of H_s, bonds counted as in the hopping
// matrix).  Every evaluation runs the single-flavour path on the 2B fields
// [s ; -s]; a local flip changes both determinants, so the local update keeps
// the two Green's functions of a chain side by side and takes the product of
// their ratios.
#include <algorithm>
#include <cmath>

#include "slq_internal.h"

namespace slq {

// out[b] = s[b], out[B + b] = -s[b] (fields of `per` spins)
__global__ void k_pair_fields(long per, int B, const int8_t* __restrict__ s, int8_t* __restrict__ out) {
  const long total = per * B;
  for (long x = (long)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (long)gridDim.x * blockDim.x) {
    const int8_t v = s[x];
    out[x] = v;
    out[total + x] = (int8_t)(-v);
  }
}

// ln phi of each field, one workgroup per field, fixed summation order
__global__ __launch_bounds__(256) void k_bare(int lx, int ly, int L, double dtJ, double kt,
                                              const int8_t* __restrict__ s_all, double* out) {
  __shared__ double red[4];
  const int N = lx * ly;
  const long b = blockIdx.x;
  const int8_t* s = s_all + b * (long)L * N;
  double acc = 0.0;
  for (long x = threadIdx.x; x < (long)L * N; x += 256) {
    const int l = (int)(x / N), i = (int)(x % N), xi = i % lx, yi = i / lx;
    const int sx = s[x];
    const int right = s[(long)l * N + (xi + 1) % lx + lx * yi];
    const int up = s[(long)l * N + xi + lx * ((yi + 1) % ly)];
    const int next = s[(long)((l + 1) % L) * N + i];
    acc += dtJ * (double)(sx * (right + up)) + kt * (double)(sx * next);
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[b] = (red[0] + red[1]) + (red[2] + red[3]);
}

// logw[b] = bare[b] + 2 (la[b] + la[B+b]); nonzero[b] = 0 when a determinant vanished
__global__ void k_bilayer_combine(int B, const double* bare, const double* la, const int8_t* sg, const int32_t* st2,
                                  double* logw, int8_t* nonzero, int32_t* status) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const bool zero = sg[b] == 0 || sg[B + b] == 0;
  logw[b] = zero ? -INFINITY : bare[b] + 2.0 * (la[b] + la[B + b]);
  if (nonzero) nonzero[b] = zero ? 0 : 1;
  if (status) status[b] |= st2[b] | st2[B + b];
}

// status[b] |= st2[b] | st2[B+b]; drift[b] = max(drift[b], d2[b], d2[B+b]) (NaN kept)
__global__ void k_pair_merge(int B, const int32_t* st2, const double* d2, int32_t* status, double* drift) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  status[b] |= st2[b] | st2[B + b];
  drift[b] = nan_max(drift[b], nan_max(d2[b], d2[B + b]));
}

// One slice of the local update of the bilayer weight, one workgroup per
// chain: for sites i = 0..N-1 in order, the ratio phi'/phi (R_a R_b)^2 from
// the two Green's functions (of s: G[b], of -s: G[B+b]), Metropolis with the
// draw at counter (i, slice, sweep, chain), and on acceptance the flip in s
// and in the paired copies and the Sherman-Morrison update
//     G <- G - x y^T,  x = (delta / R)(e_i - G[:, i]),  y = G[i, :]
// of both, delayed: the pairs (x, y) of up to FB_KD accepted flips are kept
// in X [N][KD] and Y [KD][N], the current G is G0 - X Y (its diagonal and,
// for an accepted site, its row and column are formed from G0 and the
// pairs), and G0 takes the whole rank-k update once per FB_KD flips and at
// the end of the slice.  G0 is then read and written once per FB_KD accepted
// flips instead of once per flip.
struct FlipBArgs {
  int lx, ly, L, N, B, slice;
  double a, dtJ, kt;
  int8_t* s;       // [B][L][N] the chains' fields
  int8_t* pair;    // [2B][L][N] their copies [s ; -s]
  double* G;       // [2B][N][N]
  double* X;       // [2B][N][FB_KD]
  double* Y;       // [2B][FB_KD][N]
  double* logw;    // [B]
  int64_t* accepts;
  uint64_t seed, sweep, chain0;
};

constexpr int FB_THREADS = 512;
constexpr int FB_KD = 16;

// G0 -= X Y for the k pending pairs (all threads; rows split across threads)
__device__ __forceinline__ void fb_flush(double* G0, const double* X, const double* Y, int N, int k) {
  for (long e = threadIdx.x; e < (long)N * N; e += FB_THREADS) {
    const int r = (int)(e / N), c = (int)(e - (long)r * N);
    double acc = 0.0;
    for (int q = 0; q < k; ++q) acc += X[(long)r * FB_KD + q] * Y[(long)q * N + c];
    G0[e] -= acc;
  }
}

__global__ __launch_bounds__(FB_THREADS) void k_flip_bilayer(FlipBArgs f) {
  const int N = f.N;
  const long NN = (long)N * N;
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double fa, fb, lr, gda, gdb;
  __shared__ int take;
  double* Ga = f.G + (long)b * NN;
  double* Gb = f.G + (long)(f.B + b) * NN;
  double* Xa = f.X + (long)b * N * FB_KD;
  double* Xb = f.X + (long)(f.B + b) * N * FB_KD;
  double* Ya = f.Y + (long)b * FB_KD * N;
  double* Yb = f.Y + (long)(f.B + b) * FB_KD * N;
  int8_t* s = f.s + (long)b * f.L * N;
  const int l = f.slice;
  long long acc = 0;
  int k = 0;  // pending pairs (uniform)
  for (int i = 0; i < N; ++i) {
    // the current diagonals G_ii = G0_ii - sum_q X[i][q] Y[q][i]: wave 0 for G_a, wave 1 for G_b
    if (wave < 2) {
      const double* G0 = wave == 0 ? Ga : Gb;
      const double* X = wave == 0 ? Xa : Xb;
      const double* Y = wave == 0 ? Ya : Yb;
      double v = lane < k ? X[(long)i * FB_KD + lane] * Y[(long)lane * N + i] : 0.0;
      v = wave_sum(v);
      if (lane == 0) {
        if (wave == 0) gda = G0[(long)i * N + i] - v;
        else gdb = G0[(long)i * N + i] - v;
      }
    }
    __syncthreads();
    if (tid == 0) {
      const int xi = i % f.lx, yi = i / f.lx;
      const int si = s[(long)l * N + i];
      const int nb = s[(long)l * N + (xi + 1) % f.lx + f.lx * yi] +
                     s[(long)l * N + (xi - 1 + f.lx) % f.lx + f.lx * yi] +
                     s[(long)l * N + xi + f.lx * ((yi + 1) % f.ly)] +
                     s[(long)l * N + xi + f.lx * ((yi - 1 + f.ly) % f.ly)];
      const int tn = s[(long)((l + 1) % f.L) * N + i] + s[(long)((l - 1 + f.L) % f.L) * N + i];
      const double bare = exp(-2.0 * si * (f.dtJ * nb + f.kt * tn));
      const double da = exp(2.0 * f.a * si) - 1.0, db = exp(-2.0 * f.a * si) - 1.0;
      const double ra = 1.0 + da * (1.0 - gda);
      const double rb = 1.0 + db * (1.0 - gdb);
      const double r = bare * (ra * rb) * (ra * rb);
      const double u = philox_uniform((uint64_t)i, (uint64_t)l, f.sweep, f.chain0 + b, f.seed, TAG_LOCAL);
      const int ok = u < r;
      take = ok;
      fa = da / ra;
      fb = db / rb;
      lr = ok ? log(r) : 0.0;
    }
    __syncthreads();
    if (take) {
      // new pair k of each G from the current column and row i
      const double ca = fa, cb = fb;
      for (int j = tid; j < 2 * N; j += FB_THREADS) {
        const bool second = j >= N;
        const int jj = second ? j - N : j;
        const double* G0 = second ? Gb : Ga;
        const double* X = second ? Xb : Xa;
        const double* Y = second ? Yb : Ya;
        double col = G0[(long)jj * N + i], row = G0[(long)i * N + jj];
        for (int q = 0; q < k; ++q) {
          col -= X[(long)jj * FB_KD + q] * Y[(long)q * N + i];
          row -= X[(long)i * FB_KD + q] * Y[(long)q * N + jj];
        }
        const double c = second ? cb : ca;
        double* Xw = second ? Xb : Xa;
        double* Yw = second ? Yb : Ya;
        Xw[(long)jj * FB_KD + k] = c * ((jj == i ? 1.0 : 0.0) - col);
        Yw[(long)k * N + jj] = row;
      }
      if (tid == 0) {
        const long x = (long)l * N + i;
        const int8_t v = (int8_t)(-s[x]);
        s[x] = v;
        const long per = (long)f.L * N;
        f.pair[(long)b * per + x] = v;
        f.pair[(long)(f.B + b) * per + x] = (int8_t)(-v);
        f.logw[b] += lr;
        ++acc;
      }
      ++k;
      __syncthreads();
      if (k == FB_KD) {
        fb_flush(Ga, Xa, Ya, N, k);
        fb_flush(Gb, Xb, Yb, N, k);
        k = 0;
        __syncthreads();
      }
    }
  }
  if (k > 0) {
    fb_flush(Ga, Xa, Ya, N, k);
    fb_flush(Gb, Xb, Yb, N, k);
  }
  if (tid == 0 && f.accepts) f.accepts[b] += acc;
}

static double bare_kt(double dtau, double h) { return -0.5 * std::log(std::tanh(dtau * h)); }

static int check_bilayer(const Plan& p, const slq_bilayer* bl, long batch) {
  if (!bl) {
    set_error("bilayer parameters are NULL");
    return SLQ_ERR_ARG;
  }
  if (!(bl->h > 0.0) || !std::isfinite(bl->h) || !std::isfinite(bl->J)) {
    set_error("the transverse field h must be positive and finite, J finite");
    return SLQ_ERR_ARG;
  }
  if (p.m.lx < 2 || p.m.ly < 2 || p.L < 2) {
    // (a length-1 dimension would make a spin its own neighbour in the local field)
    set_error("the bilayer workload needs lx, ly and L >= 2");
    return SLQ_ERR_ARG;
  }
  if (batch < 0) {
    set_error("batch must be >= 0");
    return SLQ_ERR_ARG;
  }
  if (2 * batch > p.max_batch) {
    set_error("the bilayer weight evaluates 2 batch fields: the plan's max_batch must be >= 2 batch");
    return SLQ_ERR_WORKSPACE;
  }
  if (p.m.chain_prec != SLQ_PREC_FP64 && p.m.chain_prec != SLQ_PREC_FP64_DENSE &&
      p.m.chain_prec != SLQ_PREC_CHECKERBOARD) {
    set_error("the bilayer workload runs FP64 chains only");
    return SLQ_ERR_ARG;
  }
  return SLQ_OK;
}

static unsigned grid_of(long n) { return (unsigned)std::max<long>(1, std::min<long>((n + 255) / 256, 4096)); }

// logw (and G of [s ; -s] when G != null) of the fields s [B]; status[B].
// The pair [s ; -s] is built in s_work (s may be its second half: each entry
// is read before the same thread writes it); ln phi is even in s and is taken
// from the first half.  Scratch: dvec [2B] (log|W|), dvec2 [B] (ln phi),
// sgn_work [2B], status2 [2B]; logw must lie outside them.
static int bilayer_eval(Plan& p, const slq_bilayer* bl, int B, const int8_t* s, double* G, double* logw,
                        int8_t* nonzero, int32_t* status, hipStream_t st) {
  const long per = (long)p.L * p.n;
  k_pair_fields<<<grid_of(per * B), 256, 0, st>>>(per, B, s, p.s_work);
  SLQ_LAUNCHED();
  int32_t* st2 = p.status2;
  SLQ_TRY(fill_i32(st2, 2 * B, 0, st));
  SLQ_TRY(launch_check_spins(p, 2 * B, p.s_work, st2, st));
  SLQ_TRY(run_chain(p, 2 * B, p.s_work, 0, st2, st));
  SLQ_TRY(launch_finish(p, 2 * B, G, p.dvec, p.sgn_work, st2, st));
  double* bare = p.dvec2;
  k_bare<<<B, 256, 0, st>>>(p.m.lx, p.m.ly, p.L, p.m.dtau * bl->J, bare_kt(p.m.dtau, bl->h), p.s_work, bare);
  SLQ_LAUNCHED();
  k_bilayer_combine<<<(B + 255) / 256, 256, 0, st>>>(B, bare, p.dvec, p.sgn_work, st2, logw, nonzero, status);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

}  // namespace slq

using namespace slq;

extern "C" {

int slq_bilayer_weight(slq_plan* plan, const slq_bilayer* bl, int32_t batch, const int8_t* d_s, double* d_logw,
                       int32_t* d_status, hipStream_t stream) {
  if (!plan) return (set_error("plan is NULL"), SLQ_ERR_ARG);
  Plan& p = plan->p;
  SLQ_TRY(check_bilayer(p, bl, batch));
  if (batch == 0) return SLQ_OK;
  if (!d_s || !d_logw) return (set_error("d_s and d_logw must not be NULL"), SLQ_ERR_ARG);
  SLQ_HIP(hipSetDevice(p.device));
  int32_t* status = d_status ? d_status : p.status;
  SLQ_TRY(fill_i32(status, batch, 0, stream));
  return bilayer_eval(p, bl, batch, d_s, nullptr, d_logw, nullptr, status, stream);
}

int slq_bilayer_green(slq_plan* plan, const slq_bilayer* bl, int32_t batch, const int8_t* d_s, double* d_G,
                      double* d_logw, int32_t* d_status, hipStream_t stream) {
  if (!plan) return (set_error("plan is NULL"), SLQ_ERR_ARG);
  Plan& p = plan->p;
  SLQ_TRY(check_bilayer(p, bl, batch));
  if (batch == 0) return SLQ_OK;
  if (!d_s || !d_G || !d_logw) return (set_error("d_s, d_G and d_logw must not be NULL"), SLQ_ERR_ARG);
  SLQ_HIP(hipSetDevice(p.device));
  int32_t* status = d_status ? d_status : p.status;
  SLQ_TRY(fill_i32(status, batch, 0, stream));
  return bilayer_eval(p, bl, batch, d_s, d_G, d_logw, nullptr, status, stream);
}

int slq_bilayer_sweep_local(slq_plan* plan, const slq_bilayer* bl, int32_t batch, int8_t* d_s, double* d_G,
                            double* d_logw, int32_t n_sweeps, uint64_t seed, uint64_t sweep0, uint64_t chain0,
                            int64_t* d_accepts, double* d_drift, int32_t* d_status, hipStream_t st) {
  if (!plan) return (set_error("plan is NULL"), SLQ_ERR_ARG);
  Plan& p = plan->p;
  SLQ_TRY(check_bilayer(p, bl, batch));
  if (n_sweeps < 0) return (set_error("n_sweeps must be >= 0"), SLQ_ERR_ARG);
  if (batch == 0 || n_sweeps == 0) return SLQ_OK;
  if (!d_s || !d_G || !d_logw) return (set_error("d_s, d_G and d_logw must not be NULL"), SLQ_ERR_ARG);
  SLQ_HIP(hipSetDevice(p.device));
  const int N = p.n, L = p.L, ns = p.m.n_stab, B = batch;
  const long per = (long)L * N, NN = (long)N * N;
  int32_t* status = d_status ? d_status : p.status;
  int64_t* acc = d_accepts ? d_accepts : p.ivec;
  double* drift = d_drift ? d_drift : p.dvec2;
  SLQ_TRY(fill_i32(status, B, 0, st));
  SLQ_TRY(fill_i64(acc, B, 0, st));
  SLQ_TRY(fill_f64(drift, B, 0.0, st));
  SLQ_TRY(launch_check_spins(p, B, d_s, status, st));
  k_pair_fields<<<grid_of(per * B), 256, 0, st>>>(per, B, d_s, p.s_work);
  SLQ_LAUNCHED();
  FlipBArgs f{};
  f.lx = p.m.lx;
  f.ly = p.m.ly;
  f.L = L;
  f.N = N;
  f.B = B;
  f.a = p.m.dtau * p.m.xi;
  f.dtJ = p.m.dtau * bl->J;
  f.kt = bare_kt(p.m.dtau, bl->h);
  f.s = d_s;
  f.pair = p.s_work;
  f.G = d_G;
  f.X = p.dX;
  f.Y = p.dY;
  f.logw = d_logw;
  f.accepts = acc;
  f.seed = seed;
  f.chain0 = chain0;
  // wrap of both Green's functions: G <- E diag(d_l) G diag(1/d_l) E^{-1}
  KronArgs k1{};
  k1.in = d_G;
  k1.strideIn = NN;
  k1.out = p.Xa;
  k1.strideOut = NN;
  k1.s = p.s_work;
  k1.count = 1;
  k1.step = 1;
  k1.scale = 1;
  k1.batch = 2 * B;
  KronArgs k2 = k1;
  k2.in = p.Xa;
  k2.out = d_G;
  k2.rows = 1;
  k2.inv = 1;
  GemmArgs w1{};
  w1.M = N;
  w1.N = N;
  w1.K = N;
  w1.A = p.E;
  w1.lda = N;
  w1.B = d_G;
  w1.ldb = N;
  w1.strideB = NN;
  w1.C = p.Xa;
  w1.ldc = N;
  w1.strideC = NN;
  w1.S = p.s_work;
  w1.strideS = per;
  w1.consts = p.consts;
  w1.alpha = 1.0;
  w1.batch = 2 * B;
  GemmArgs w2 = w1;
  w2.A = p.Xa;
  w2.strideA = NN;
  w2.B = p.Einv;
  w2.strideB = 0;
  w2.C = d_G;
  w2.inv_scale = 1;
  for (int k = 0; k < n_sweeps; ++k) {
    f.sweep = sweep0 + k;
    for (int l = 1; l <= L; ++l) {
      f.slice = l - 1;
      k_flip_bilayer<<<B, FB_THREADS, 0, st>>>(f);
      SLQ_LAUNCHED();
      if (has_structured(p)) {
        k1.slice0 = l - 1;
        k2.slice0 = l - 1;
        SLQ_TRY(launch_kron(p, k1, st));
        SLQ_TRY(launch_kron(p, k2, st));
      } else {
        w1.slice = l - 1;
        w2.slice = l - 1;
        SLQ_TRY(launch_gemm(w1, false, false, st));
        SLQ_TRY(launch_gemm(w2, false, false, st));
      }
      if (l % ns == 0) {
        // both Green's functions afresh from the cyclic chain that ends at B_l
        SLQ_TRY(fill_i32(p.status2, 2 * B, 0, st));
        SLQ_TRY(run_chain(p, 2 * B, p.s_work, l % L, p.status2, st));
        SLQ_TRY(launch_finish(p, 2 * B, p.Xa, p.dvec, p.sgn_work, p.status2, st));
        SLQ_TRY(fill_f64(p.dvec, 2 * B, 0.0, st));
        SLQ_TRY(launch_drift(p, 2 * B, d_G, p.Xa, p.dvec, p.status2, st));
        k_pair_merge<<<(B + 255) / 256, 256, 0, st>>>(B, p.status2, p.dvec, status, drift);
        SLQ_LAUNCHED();
      }
    }
  }
  return SLQ_OK;
}

int slq_bilayer_cumulative_step(slq_plan* plan, const slq_eff* eff, const slq_bilayer* bl, int32_t batch,
                                int8_t* d_s, double* d_logw, int32_t n_moves, uint64_t seed, uint64_t step,
                                uint64_t chain0, int8_t* d_accepted, double* d_logA, int32_t* d_status,
                                hipStream_t stream) {
  if (!plan || !eff || !d_s || !d_logw) return (set_error("NULL argument"), SLQ_ERR_ARG);
  Plan& p = plan->p;
  const Eff& e = eff->e;
  if (e.plan != &p) return (set_error("eff belongs to another plan"), SLQ_ERR_ARG);
  SLQ_TRY(check_bilayer(p, bl, batch));
  if (batch == 0) return SLQ_OK;
  if (n_moves < 0) return (set_error("n_moves must be >= 0"), SLQ_ERR_ARG);
  SLQ_HIP(hipSetDevice(p.device));
  const int B = batch;
  const long per = (long)p.L * p.n;
  int32_t* status = d_status ? d_status : p.status;
  SLQ_TRY(fill_i32(status, B, 0, stream));
  SLQ_TRY(launch_check_spins(p, B, d_s, status, stream));
  // the proposal s' in the second half of s_work: effective moves, features,
  // then the pair [s' ; -s'] in s_work, so that s' ends in its first half
  int8_t* prop = p.s_work + per * B;
  SLQ_TRY(copy_i8(d_s, prop, per * B, stream));
  SLQ_TRY(launch_eff_sweep(p, e, B, prop, n_moves, seed, step, chain0, nullptr, nullptr, stream));
  SLQ_TRY(launch_features(p, e, B, d_s, p.F_old, stream));
  SLQ_TRY(launch_features(p, e, B, prop, p.F_new, stream));
  double *sn_old = nullptr, *sn_new = nullptr;
  if (e.net_on) SLQ_TRY(net_pair(p, e, B, d_s, prop, &sn_old, &sn_new, stream));
  double* new_logw = p.dvec2 + B;
  int8_t* nonzero = p.sgn_work2;
  SLQ_TRY(bilayer_eval(p, bl, B, prop, nullptr, new_logw, nonzero, status, stream));
  // omega > 0: the sign array Eq. 4's acceptance keeps is a dummy here
  return launch_accept(p, e, B, d_s, p.s_work, d_logw, p.sgn_work2 + B, new_logw, nonzero, p.F_old, p.F_new,
                       sn_old, sn_new, seed, step, chain0, d_accepted, d_logA, stream);
}

}  // extern "C"
