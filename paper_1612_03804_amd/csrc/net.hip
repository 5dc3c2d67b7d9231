// Learned effective action: a small convolutional network added to the
// linear effective model ("Formalism of SLDQMC": the "..." of Eq. 2,
// interactions beyond the pair couplings), trained on the device and used in
// the effective moves of cumulative updates.
//
//   a1[c]  = b1[c] + sum_{k in 3^3} W1[c][k] s(x + o(k))             c = 0..7
//   h1     = tanh(a1)
//   a2[c]  = b2[c] + sum_{c', k} W2[c][c'][k] h1[c'](x + o(k))
//   h2     = tanh(a2)
//   S_net  = b3 + sum_c w3[c] sum_x h2[c](x)
// with o(k) = (k/9 - 1, (k/3)%3 - 1, k%3 - 1) along (time, y, x), all three
// axes periodic.  Parameters (1969): W1[8][27], b1[8], W2[8][8][27], b2[8],
// w3[8], b3.  Arithmetic in FP32 (production) or FP64 (T = double).
//
// Training minimises (1/B) sum_b (S_net(s_b) - r_b)^2 with r_b = y_b - S_lin(s_b)
// (the residual of the linear model) by Adam.  All reductions have a fixed
// order, so the gradient is deterministic.
#include <algorithm>
#include <cmath>

#include "slq_internal.h"

namespace slq {

constexpr int NC = 8;
constexpr int P_W1 = 0, P_B1 = 216, P_W2 = 224, P_B2 = 1952, P_W3 = 1960, P_B3 = 1968;
constexpr int NET_BLOCK = 256;
constexpr int WG_CHUNKS = 32;  // site chunks per sample in the weight-gradient reduction

struct NetDims {
  int L, ly, lx;
  long LN;
};

__device__ __forceinline__ int wrapi(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}
__device__ __forceinline__ long nb_site(const NetDims& d, int t, int y, int x, int k) {
  return ((long)wrapi(t + k / 9 - 1, d.L) * d.ly + wrapi(y + (k / 3) % 3 - 1, d.ly)) * d.lx + wrapi(x + k % 3 - 1, d.lx);
}
template <typename T>
__device__ __forceinline__ T wsum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------- forward ----
template <typename T>
__global__ __launch_bounds__(NET_BLOCK) void k_net_l1(NetDims d, const int8_t* __restrict__ s_all,
                                                     const double* __restrict__ prm, T* __restrict__ a1,
                                                     T* __restrict__ h1) {
  __shared__ T W[224];
  for (int i = threadIdx.x; i < 224; i += NET_BLOCK) W[i] = (T)prm[i];
  __syncthreads();
  const long b = blockIdx.y;
  const long x0 = (long)blockIdx.x * NET_BLOCK + threadIdx.x;
  if (x0 >= d.LN) return;
  const int8_t* s = s_all + b * d.LN;
  const int t = (int)(x0 / ((long)d.ly * d.lx)), y = (int)((x0 / d.lx) % d.ly), x = (int)(x0 % d.lx);
  T acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = W[P_B1 + c];
  for (int k = 0; k < 27; ++k) {
    const T v = (T)s[nb_site(d, t, y, x, k)];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] += W[c * 27 + k] * v;
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    a1[(b * NC + c) * d.LN + x0] = acc[c];
    h1[(b * NC + c) * d.LN + x0] = tanh(acc[c]);
  }
}

// a2, h2 and per-block pooled sums part[b][blk][c] of h2.
template <typename T>
__global__ __launch_bounds__(NET_BLOCK) void k_net_l2(NetDims d, const double* __restrict__ prm,
                                                     const T* __restrict__ h1, T* __restrict__ a2,
                                                     T* __restrict__ h2, T* __restrict__ part) {
  __shared__ T W2[NC * NC * 27 + NC];
  __shared__ T red[NC][NET_BLOCK / 64];
  for (int i = threadIdx.x; i < NC * NC * 27 + NC; i += NET_BLOCK) W2[i] = (T)prm[P_W2 + i];
  __syncthreads();
  const long b = blockIdx.y;
  const long x0 = (long)blockIdx.x * NET_BLOCK + threadIdx.x;
  const bool ok = x0 < d.LN;
  T h[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) h[c] = (T)0;
  if (ok) {
    const int t = (int)(x0 / ((long)d.ly * d.lx)), y = (int)((x0 / d.lx) % d.ly), x = (int)(x0 % d.lx);
    T acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = W2[NC * NC * 27 + c];
    for (int k = 0; k < 27; ++k) {
      const long nb = nb_site(d, t, y, x, k);
#pragma unroll
      for (int cp = 0; cp < NC; ++cp) {
        const T v = h1[(b * NC + cp) * d.LN + nb];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += W2[(c * NC + cp) * 27 + k] * v;
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      a2[(b * NC + c) * d.LN + x0] = acc[c];
      h[c] = tanh(acc[c]);
      h2[(b * NC + c) * d.LN + x0] = h[c];
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const T v = wsum(h[c]);
    if (lane == 0) red[c][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < NC) {
    T tot = (T)0;
    for (int w = 0; w < NET_BLOCK / 64; ++w) tot += red[threadIdx.x][w];
    part[(b * gridDim.x + blockIdx.x) * NC + threadIdx.x] = tot;
  }
}

// S[b] = b3 + sum_c w3[c] pool[b][c]; pool from the block partials in order.
template <typename T>
__global__ void k_net_pool(int nblk, const double* __restrict__ prm, const T* __restrict__ part, T* __restrict__ pool,
                           double* __restrict__ S) {
  __shared__ double pc[NC];
  const long b = blockIdx.x;
  if (threadIdx.x < NC) {
    T tot = (T)0;
    for (int k = 0; k < nblk; ++k) tot += part[(b * nblk + k) * NC + threadIdx.x];
    pool[b * NC + threadIdx.x] = tot;
    pc[threadIdx.x] = (double)tot;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = prm[P_B3];
    for (int c = 0; c < NC; ++c) v += prm[P_W3 + c] * pc[c];
    S[b] = v;
  }
}

// ------------------------------------------------------------ backward ----
// gS[b] = 2 (S_b - r_b) / B with r_b = y_b - (c0 + sum_k lambda_k F[b][k]); loss in out[0]
__global__ void k_net_residual(int B, int K, const double* __restrict__ S, const double* __restrict__ y,
                               const double* __restrict__ theta, const double* __restrict__ F, double* __restrict__ gS,
                               double* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double l = 0.0;
  for (int b = 0; b < B; ++b) {
    double lin = theta[0];
    for (int k = 0; k < K; ++k) lin += theta[1 + k] * F[(long)b * K + k];
    const double r = S[b] - (y[b] - lin);
    gS[b] = 2.0 * r / B;
    l += r * r / B;
  }
  if (loss) loss[0] = l;
}

// dz2 = gS w3 (1 - h2^2)
template <typename T>
__global__ __launch_bounds__(NET_BLOCK) void k_net_dz2(NetDims d, const double* __restrict__ prm,
                                                      const double* __restrict__ gS, const T* __restrict__ h2,
                                                      T* __restrict__ dz2) {
  const long b = blockIdx.y;
  const long x0 = (long)blockIdx.x * NET_BLOCK + threadIdx.x;
  if (x0 >= d.LN) return;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const long o = (b * NC + c) * d.LN + x0;
    const T h = h2[o];
    dz2[o] = (T)(gS[b] * prm[P_W3 + c]) * ((T)1 - h * h);
  }
}

// dz1[c'](y) = (1 - h1^2) sum_{c,k} W2[c][c'][k] dz2[c](y - o(k))
template <typename T>
__global__ __launch_bounds__(NET_BLOCK) void k_net_dz1(NetDims d, const double* __restrict__ prm,
                                                      const T* __restrict__ h1, const T* __restrict__ dz2,
                                                      T* __restrict__ dz1) {
  __shared__ T W2[NC * NC * 27];
  for (int i = threadIdx.x; i < NC * NC * 27; i += NET_BLOCK) W2[i] = (T)prm[P_W2 + i];
  __syncthreads();
  const long b = blockIdx.y;
  const long x0 = (long)blockIdx.x * NET_BLOCK + threadIdx.x;
  if (x0 >= d.LN) return;
  const int t = (int)(x0 / ((long)d.ly * d.lx)), y = (int)((x0 / d.lx) % d.ly), x = (int)(x0 % d.lx);
  T acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = (T)0;
  for (int k = 0; k < 27; ++k) {
    const long src = nb_site(d, t, y, x, 26 - k);  // y - o(k) = y + o(26 - k)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const T g = dz2[(b * NC + c) * d.LN + src];
#pragma unroll
      for (int cp = 0; cp < NC; ++cp) acc[cp] += W2[(c * NC + cp) * 27 + k] * g;
    }
  }
#pragma unroll
  for (int cp = 0; cp < NC; ++cp) {
    const long o = (b * NC + cp) * d.LN + x0;
    const T h = h1[o];
    dz1[o] = acc[cp] * ((T)1 - h * h);
  }
}

// Partial weight gradients of W1, b1, W2, b2 over one chunk of one sample.
template <typename T>
__global__ __launch_bounds__(NET_BLOCK) void k_net_wgrad(NetDims d, const int8_t* __restrict__ s_all,
                                                        const T* __restrict__ h1, const T* __restrict__ dz1,
                                                        const T* __restrict__ dz2, double* __restrict__ part) {
  const long b = blockIdx.y;
  const int chunk = blockIdx.x;
  const long per = (d.LN + WG_CHUNKS - 1) / WG_CHUNKS;
  const long beg = chunk * per, end = std::min<long>(d.LN, beg + per);
  const int8_t* s = s_all + b * d.LN;
  constexpr int NP = P_W3;  // 1960 parameters handled here
  constexpr int PPT = (NP + NET_BLOCK - 1) / NET_BLOCK;
  T acc[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) acc[q] = (T)0;
  for (long x0 = beg; x0 < end; ++x0) {
    const int t = (int)(x0 / ((long)d.ly * d.lx)), y = (int)((x0 / d.lx) % d.ly), x = (int)(x0 % d.lx);
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int p = threadIdx.x + q * NET_BLOCK;
      if (p < P_B1) {  // W1[c][k]
        const int c = p / 27, k = p % 27;
        acc[q] += dz1[(b * NC + c) * d.LN + x0] * (T)s[nb_site(d, t, y, x, k)];
      } else if (p < P_W2) {  // b1[c]
        acc[q] += dz1[(b * NC + (p - P_B1)) * d.LN + x0];
      } else if (p < P_B2) {  // W2[c][c'][k]
        const int r = p - P_W2, c = r / (NC * 27), cp = (r / 27) % NC, k = r % 27;
        acc[q] += dz2[(b * NC + c) * d.LN + x0] * h1[(b * NC + cp) * d.LN + nb_site(d, t, y, x, k)];
      } else if (p < NP) {  // b2[c]
        acc[q] += dz2[(b * NC + (p - P_B2)) * d.LN + x0];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int p = threadIdx.x + q * NET_BLOCK;
    if (p < NP) part[((long)b * WG_CHUNKS + chunk) * NP + p] = (double)acc[q];
  }
}

// grad[p] = fixed-order sum of the partials; w3 and b3 from the pools.
template <typename T>
__global__ void k_net_reduce(int B, const double* __restrict__ part, const T* __restrict__ pool,
                             const double* __restrict__ gS, double* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= SLQ_NET_PARAMS) return;
  double tot = 0.0;
  if (p < P_W3) {
    for (long k = 0; k < (long)B * WG_CHUNKS; ++k) tot += part[k * P_W3 + p];
  } else if (p < P_B3) {
    for (int b = 0; b < B; ++b) tot += gS[b] * (double)pool[(long)b * NC + (p - P_W3)];
  } else {
    for (int b = 0; b < B; ++b) tot += gS[b];
  }
  grad[p] = tot;
}

// Adam (Kingma & Ba 2015) with bias correction, step t >= 1.
__global__ void k_adam(int n, double* __restrict__ prm, const double* __restrict__ g, double* __restrict__ m,
                       double* __restrict__ v, double t, double lr, double b1, double b2, double eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
  const double mm = b1 * m[p] + (1.0 - b1) * g[p];
  const double vv = b2 * v[p] + (1.0 - b2) * g[p] * g[p];
  m[p] = mm;
  v[p] = vv;
  prm[p] -= lr * (mm / c1) / (sqrt(vv / c2) + eps);
}

// ---------------------------------------------------------- workspace ----
struct NetWork {
  long LN = 0;
  int batch = 0;
  int nblk = 0;
  void* base = nullptr;
  size_t bytes = 0;
  double *a1, *h1, *a2, *h2, *dz1, *dz2;  // typed buffers, sized for FP64
  double* part;                           // l2 block partials [batch][nblk][8]
  double* pool;                           // [batch][8]
  double* wpart;                          // [batch][WG_CHUNKS][1960]
  double *S, *S2, *gS, *F;                // [batch], [batch], [batch], [batch][64]
};

static NetWork& net_work(Plan& p) {
  static_assert(sizeof(NetWork) > 0, "");
  return *reinterpret_cast<NetWork*>(p.net_state);
}

// Layout of the network buffers for max_batch fields (in doubles); with d
// set, w's pointers are placed.
static size_t net_layout(const Plan& p, NetWork* w, double* d) {
  const long LN = (long)p.L * p.n;
  const int nblk = (int)((LN + NET_BLOCK - 1) / NET_BLOCK);
  const long B = p.max_batch, act = (long)NC * LN * B;
  size_t off = 0;
  auto take = [&](size_t n) {
    const size_t o = off;
    off += (n + 31) / 32 * 32;
    return o;
  };
  const size_t o1 = take(act), o2 = take(act), o3 = take(act), o4 = take(act), o5 = take(act), o6 = take(act);
  const size_t op = take((size_t)B * nblk * NC), opl = take(B * NC), ow = take((size_t)B * WG_CHUNKS * P_W3);
  const size_t oS = take(B), oS2 = take(B), og = take(B), oF = take(B * 64);
  if (w && d) {
    w->LN = LN;
    w->batch = (int)B;
    w->nblk = nblk;
    w->base = d;
    w->bytes = off * sizeof(double);
    w->a1 = d + o1;
    w->h1 = d + o2;
    w->a2 = d + o3;
    w->h2 = d + o4;
    w->dz1 = d + o5;
    w->dz2 = d + o6;
    w->part = d + op;
    w->pool = d + opl;
    w->wpart = d + ow;
    w->S = d + oS;
    w->S2 = d + oS2;
    w->gS = d + og;
    w->F = d + oF;
  }
  return off;
}

size_t net_bytes_for(const Plan& p) { return sizeof(double) * net_layout(p, nullptr, nullptr); }

int bind_net(Plan& p) {
  if (p.net_state) return SLQ_OK;
  NetWork* w = new (std::nothrow) NetWork();
  if (!w) {
    set_error("host allocation failed");
    return SLQ_ERR_DEVICE;
  }
  net_layout(p, w, (double*)p.net_base);
  p.net_state = w;
  return SLQ_OK;
}

static int ensure_net(Plan& p) {
  if (p.net_state) return SLQ_OK;
  set_error("the plan was created without SLQ_PLAN_NET (no room for the network's activations)");
  return SLQ_ERR_WORKSPACE;
}

void release_net(Plan& p) {
  if (!p.net_state) return;
  delete reinterpret_cast<NetWork*>(p.net_state);
  p.net_state = nullptr;
}

static NetDims dims_of(const Plan& p) { return NetDims{p.L, p.m.ly, p.m.lx, (long)p.L * p.n}; }

// Forward pass: activations into the workspace, S_net into S.
template <typename T>
static int forward_t(Plan& p, int batch, const int8_t* s, const double* prm, double* S, hipStream_t st) {
  NetWork& w = net_work(p);
  const NetDims d = dims_of(p);
  dim3 grid(w.nblk, batch);
  k_net_l1<T><<<grid, NET_BLOCK, 0, st>>>(d, s, prm, (T*)w.a1, (T*)w.h1);
  SLQ_LAUNCHED();
  k_net_l2<T><<<grid, NET_BLOCK, 0, st>>>(d, prm, (const T*)w.h1, (T*)w.a2, (T*)w.h2, (T*)w.part);
  SLQ_LAUNCHED();
  k_net_pool<T><<<batch, 64, 0, st>>>(w.nblk, prm, (const T*)w.part, (T*)w.pool, S);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

int net_forward(Plan& p, int prec, int batch, const int8_t* s, const double* prm, double* S, hipStream_t st) {
  int rc = ensure_net(p);
  if (rc != SLQ_OK) return rc;
  return prec == SLQ_PREC_FP64 ? forward_t<double>(p, batch, s, prm, S, st) : forward_t<float>(p, batch, s, prm, S, st);
}

template <typename T>
static int gradient_t(Plan& p, const Eff& e, int batch, const int8_t* s, const double* y, const double* prm,
                      double* grad, double* loss, hipStream_t st) {
  NetWork& w = net_work(p);
  const NetDims d = dims_of(p);
  int rc = forward_t<T>(p, batch, s, prm, w.S, st);
  if (rc != SLQ_OK) return rc;
  rc = launch_features(p, e, batch, s, w.F, st);
  if (rc != SLQ_OK) return rc;
  k_net_residual<<<1, 64, 0, st>>>(batch, e.n_terms, w.S, y, e.d_theta, w.F, w.gS, loss);
  SLQ_LAUNCHED();
  dim3 grid(w.nblk, batch);
  k_net_dz2<T><<<grid, NET_BLOCK, 0, st>>>(d, prm, w.gS, (const T*)w.h2, (T*)w.dz2);
  SLQ_LAUNCHED();
  k_net_dz1<T><<<grid, NET_BLOCK, 0, st>>>(d, prm, (const T*)w.h1, (const T*)w.dz2, (T*)w.dz1);
  SLQ_LAUNCHED();
  k_net_wgrad<T><<<dim3(WG_CHUNKS, batch), NET_BLOCK, 0, st>>>(d, s, (const T*)w.h1, (const T*)w.dz1,
                                                               (const T*)w.dz2, w.wpart);
  SLQ_LAUNCHED();
  k_net_reduce<T><<<(SLQ_NET_PARAMS + 255) / 256, 256, 0, st>>>(batch, w.wpart, (const T*)w.pool, w.gS, grad);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

// -------------------------------------------------- moves with the net ----
// Effective moves under S_lin + S_net.  Classes: one slice and one colour of
// the greedy colouring of the graph that also links sites within spatial
// Chebyshev distance 4 (a flip changes h2 within distance 2), so the
// neighbourhoods touched by two sites of a class are disjoint.  The network
// state (a1, h1, a2 of the current field) is kept and updated locally on
// every accepted flip; one wavefront evaluates one site.
struct NetMoveArgs {
  NetDims d;
  const double* prm;
  const int32_t* col_sites;
  const int32_t* col_off;
  int n_colours;
  int n_moves;
  uint64_t seed, step, chain0;
  int64_t* accepts;
  double* dS_out;
};

constexpr int NM_THREADS = 512;
constexpr int NM_WAVES = NM_THREADS / 64;

template <typename T>
__global__ __launch_bounds__(NM_THREADS) void k_eff_sweep_net(EffDev ed, NetMoveArgs a, int8_t* s_all, T* a1_all,
                                                             T* h1_all, T* a2_all) {
  __shared__ T W1[216], W2[NC * NC * 27], w3[NC];
  __shared__ T dh1[NM_WAVES][NC * 27], na1[NM_WAVES][NC * 27], na2[NM_WAVES][NC * 125];
  __shared__ double redd[NM_WAVES];
  __shared__ long long redi[NM_WAVES];
  for (int i = threadIdx.x; i < 216; i += NM_THREADS) W1[i] = (T)a.prm[P_W1 + i];
  for (int i = threadIdx.x; i < NC * NC * 27; i += NM_THREADS) W2[i] = (T)a.prm[P_W2 + i];
  if (threadIdx.x < NC) w3[threadIdx.x] = (T)a.prm[P_W3 + threadIdx.x];
  __syncthreads();
  const NetDims& d = a.d;
  const long b = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int8_t* s = s_all + b * d.LN;
  T* A1 = a1_all + b * NC * d.LN;
  T* H1 = h1_all + b * NC * d.LN;
  T* A2 = a2_all + b * NC * d.LN;
  const uint64_t chain = a.chain0 + b;
  const int n_classes = a.n_colours * d.L;
  long long acc = 0;
  double dsum = 0.0;
  for (int mv = 0; mv < a.n_moves; ++mv) {
    const uint32_t cls = philox_below((uint32_t)n_classes, 0, (uint64_t)mv, a.step, chain, a.seed, TAG_EFFECTIVE);
    const int colour = (int)(cls % a.n_colours);
    const int l = (int)(cls / a.n_colours);
    const int beg = a.col_off[colour], end = a.col_off[colour + 1];
    for (int q = beg + wave; q < end; q += NM_WAVES) {
      const int i = a.col_sites[q];
      const int yy = i / d.lx, xx = i % d.lx;
      const long xs = (long)l * ed.N + i;
      const double sx = (double)s[xs];
      // linear part: lanes split the terms
      double hs = 0.0;
      for (int k = lane; k < ed.n_terms; k += 64) hs += ed.theta[1 + k] * (double)local_field_dev(ed, s, k, i, l);
      hs = wave_sum(hs);
      // layer-1 change on the 27 sites y = x + o(e): a1 gains W1[c][26 - e] (-2 s_x)
      for (int j = lane; j < NC * 27; j += 64) {
        const int c = j / 27, e = j % 27;
        const long y = nb_site(d, l, yy, xx, e);
        const T an = A1[(long)c * d.LN + y] + W1[c * 27 + (26 - e)] * (T)(-2.0 * sx);
        na1[wave][j] = an;
        dh1[wave][j] = tanh(an) - H1[(long)c * d.LN + y];
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      // layer-2 change on the 125 sites z = x + g, |g| <= 2
      T dnet = (T)0;
      for (int j = lane; j < NC * 125; j += 64) {
        const int c = j / 125, gi = j % 125;
        const int gt = gi / 25 - 2, gy = (gi / 5) % 5 - 2, gx = gi % 5 - 2;
        T da = (T)0;
        for (int e = 0; e < 27; ++e) {
          const int ft = e / 9 - 1 - gt, fy = (e / 3) % 3 - 1 - gy, fx = e % 3 - 1 - gx;
          if (ft < -1 || ft > 1 || fy < -1 || fy > 1 || fx < -1 || fx > 1) continue;
          const int kf = (ft + 1) * 9 + (fy + 1) * 3 + (fx + 1);
#pragma unroll
          for (int cp = 0; cp < NC; ++cp) da += W2[(c * NC + cp) * 27 + kf] * dh1[wave][cp * 27 + e];
        }
        const long z = ((long)wrapi(l + gt, d.L) * d.ly + wrapi(yy + gy, d.ly)) * d.lx + wrapi(xx + gx, d.lx);
        const T ao = A2[(long)c * d.LN + z];
        const T an = ao + da;
        na2[wave][j] = an;
        dnet += w3[c] * (tanh(an) - tanh(ao));
      }
      const double dS = -2.0 * sx * hs + (double)wsum(dnet);
      const double u = philox_uniform((uint64_t)(1 + xs), (uint64_t)mv, a.step, chain, a.seed, TAG_EFFECTIVE);
      const bool take = u < exp(dS);
      if (take) {
        for (int j = lane; j < NC * 27; j += 64) {
          const int c = j / 27, e = j % 27;
          const long y = nb_site(d, l, yy, xx, e);
          A1[(long)c * d.LN + y] = na1[wave][j];
          H1[(long)c * d.LN + y] = tanh(na1[wave][j]);
        }
        for (int j = lane; j < NC * 125; j += 64) {
          const int c = j / 125, gi = j % 125;
          const int gt = gi / 25 - 2, gy = (gi / 5) % 5 - 2, gx = gi % 5 - 2;
          const long z = ((long)wrapi(l + gt, d.L) * d.ly + wrapi(yy + gy, d.ly)) * d.lx + wrapi(xx + gx, d.lx);
          A2[(long)c * d.LN + z] = na2[wave][j];
        }
        if (lane == 0) {
          s[xs] = (int8_t)(-s[xs]);
          ++acc;
          dsum += dS;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
  }
  long long a2v = acc;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a2v += __shfl_xor(a2v, o, 64);
  dsum = wave_sum(dsum);
  if (lane == 0) {
    redi[wave] = a2v;
    redd[wave] = dsum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long ta = 0;
    double td = 0.0;
    for (int w2 = 0; w2 < NM_WAVES; ++w2) {
      ta += redi[w2];
      td += redd[w2];
    }
    if (a.accepts) a.accepts[b] = ta;
    if (a.dS_out) a.dS_out[b] = td;
  }
}

int launch_eff_sweep_net(Plan& p, const Eff& e, int batch, int8_t* s, int n_moves, uint64_t seed, uint64_t step,
                         uint64_t chain0, int64_t* accepts, double* dS, hipStream_t st) {
  int rc = ensure_net(p);
  if (rc != SLQ_OK) return rc;
  NetWork& w = net_work(p);
  // the state of the incoming fields
  rc = net_forward(p, e.net_prec, batch, s, e.d_net, w.S, st);
  if (rc != SLQ_OK) return rc;
  NetMoveArgs a;
  a.d = dims_of(p);
  a.prm = e.d_net;
  a.col_sites = e.d_ncol_sites;
  a.col_off = e.d_ncol_off;
  a.n_colours = e.n_ncolours;
  a.n_moves = n_moves;
  a.seed = seed;
  a.step = step;
  a.chain0 = chain0;
  a.accepts = accepts;
  a.dS_out = dS;
  const EffDev ed = eff_dev_view(p, e);
  // FP64 state only (slq_eff_set_net refuses other precisions for proposals)
  k_eff_sweep_net<double><<<batch, NM_THREADS, 0, st>>>(ed, a, s, w.a1, w.h1, w.a2);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

// S_net of the incoming fields (into *old) and of the proposals (into *neu)
int net_pair(Plan& p, const Eff& e, int batch, const int8_t* s_old, const int8_t* s_new, double** old_out,
             double** new_out, hipStream_t st) {
  int rc = ensure_net(p);
  if (rc != SLQ_OK) return rc;
  NetWork& w = net_work(p);
  rc = net_forward(p, e.net_prec, batch, s_old, e.d_net, w.S, st);
  if (rc == SLQ_OK) rc = net_forward(p, e.net_prec, batch, s_new, e.d_net, w.S2, st);
  *old_out = w.S;
  *new_out = w.S2;
  return rc;
}

}  // namespace slq

using namespace slq;

extern "C" {

int slq_net_forward(slq_plan* plan, int32_t net_prec, int32_t batch, const int8_t* d_s, const double* d_params,
                    double* d_S, hipStream_t stream) {
  if (!plan || !d_s || !d_params || !d_S) {
    set_error("NULL argument");
    return SLQ_ERR_ARG;
  }
  Plan& p = plan->p;
  if (batch < 0 || batch > p.max_batch) {
    set_error("batch must be in [0, max_batch]");
    return batch < 0 ? SLQ_ERR_ARG : SLQ_ERR_WORKSPACE;
  }
  if (net_prec != SLQ_PREC_FP64 && net_prec != SLQ_PREC_FP32) {
    set_error("net_prec must be SLQ_PREC_FP64 or SLQ_PREC_FP32");
    return SLQ_ERR_ARG;
  }
  if (batch == 0) return SLQ_OK;
  SLQ_HIP(hipSetDevice(p.device));
  return net_forward(p, net_prec, batch, d_s, d_params, d_S, stream);
}

int slq_net_gradient(slq_plan* plan, const slq_eff* eff, int32_t net_prec, int32_t batch, const int8_t* d_s,
                     const double* d_y, const double* d_params, double* d_grad, double* d_loss, hipStream_t stream) {
  if (!plan || !eff || !d_s || !d_y || !d_params || !d_grad) {
    set_error("NULL argument");
    return SLQ_ERR_ARG;
  }
  Plan& p = plan->p;
  if (eff->e.plan != &p) {
    set_error("eff belongs to another plan");
    return SLQ_ERR_ARG;
  }
  if (batch < 1 || batch > p.max_batch) {
    set_error("batch must be in [1, max_batch]");
    return batch < 1 ? SLQ_ERR_ARG : SLQ_ERR_WORKSPACE;
  }
  if (net_prec != SLQ_PREC_FP64 && net_prec != SLQ_PREC_FP32) {
    set_error("net_prec must be SLQ_PREC_FP64 or SLQ_PREC_FP32");
    return SLQ_ERR_ARG;
  }
  SLQ_HIP(hipSetDevice(p.device));
  int rc = ensure_net(p);
  if (rc != SLQ_OK) return rc;
  return net_prec == SLQ_PREC_FP64
             ? gradient_t<double>(p, eff->e, batch, d_s, d_y, d_params, d_grad, d_loss, stream)
             : gradient_t<float>(p, eff->e, batch, d_s, d_y, d_params, d_grad, d_loss, stream);
}

int slq_net_adam(int32_t n, double* d_params, const double* d_grad, double* d_m, double* d_v, int64_t t, double lr,
                 double beta1, double beta2, double eps, hipStream_t stream) {
  if (!d_params || !d_grad || !d_m || !d_v || n < 1 || t < 1) {
    set_error("bad argument");
    return SLQ_ERR_ARG;
  }
  k_adam<<<(n + 255) / 256, 256, 0, stream>>>(n, d_params, d_grad, d_m, d_v, (double)t, lr, beta1, beta2, eps);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

}  // extern "C"
