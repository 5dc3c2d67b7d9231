// Equal-time measurements from the Green's function G_ij = <c_i c_j^dag> of
// one configuration (the fermions are free for a given field, so Wick's
// theorem gives every equal-time expectation from G):
//     <c_i^dag c_j> = delta_ij - G_ji,
//     <n_i n_j>     = (1 - G_ii)(1 - G_jj) + (delta_ij - G_ji) G_ij.
// Per field: the density, the hopping energy per site and the staggered
// density correlation S(pi, pi).  One workgroup per field; every sum has a
// fixed partition over threads and a fixed combination order.
#include <algorithm>

#include "slq_internal.h"

namespace slq {

constexpr int ME_THREADS = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(ME_THREADS) void k_equal_time(int lx, int ly, double t, const double* __restrict__ Gall,
                                                           double* out) {
  __shared__ double red[ME_THREADS / 64];
  const int N = lx * ly;
  const long b = blockIdx.x;
  const double* G = Gall + b * (long)N * N;
  double dens = 0.0, hop = 0.0, stag = 0.0, diag = 0.0;
  for (int i = threadIdx.x; i < N; i += ME_THREADS) {
    const int x = i % lx, y = i / lx;
    const double gii = G[(long)i * N + i];
    const double sg = ((x + y) & 1) ? -1.0 : 1.0;
    dens += 1.0 - gii;
    stag += sg * (1.0 - gii);
    diag += gii;
    // bonds to +x and +y, each counted once per site (a length-2 side lists a pair twice)
    const int jx = (x + 1) % lx + lx * y, jy = x + lx * ((y + 1) % ly);
    if (jx != i) hop += t * (G[(long)i * N + jx] + G[(long)jx * N + i]);
    if (jy != i) hop += t * (G[(long)i * N + jy] + G[(long)jy * N + i]);
  }
  // sum_ij s_i s_j G_ji G_ij over (i, j) pairs split across threads
  double cross = 0.0;
  for (long e = threadIdx.x; e < (long)N * N; e += ME_THREADS) {
    const int i = (int)(e / N), j = (int)(e % N);
    const double si = (((i % lx) + (i / lx)) & 1) ? -1.0 : 1.0;
    const double sj = (((j % lx) + (j / lx)) & 1) ? -1.0 : 1.0;
    cross += si * sj * G[(long)j * N + i] * G[e];
  }
  dens = block_sum(dens, red);
  hop = block_sum(hop, red);
  stag = block_sum(stag, red);
  diag = block_sum(diag, red);
  cross = block_sum(cross, red);
  if (threadIdx.x == 0) {
    out[3 * b + 0] = dens / N;
    out[3 * b + 1] = hop / N;
    out[3 * b + 2] = (stag * stag + diag - cross) / N;
  }
}

}  // namespace slq

using namespace slq;

extern "C" int slq_measure_equal_time(slq_plan* plan, int32_t batch, const double* d_G, double* d_out,
                                      hipStream_t stream) {
  if (!plan || !d_G || !d_out) {
    set_error("NULL argument");
    return SLQ_ERR_ARG;
  }
  Plan& p = plan->p;
  if (batch < 0) {
    set_error("batch must be >= 0");
    return SLQ_ERR_ARG;
  }
  if (batch == 0) return SLQ_OK;
  SLQ_HIP(hipSetDevice(p.device));
  k_equal_time<<<batch, ME_THREADS, 0, stream>>>(p.m.lx, p.m.ly, p.m.t, d_G, d_out);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

namespace slq {

// X <- B_{l1} ... B_{l0+1} X (slices l0+1 .. l1 of the chain, 0-based l0 .. l1-1)
static int chain_apply(Plan& p, int batch, const int8_t* s, int l0, int l1, const double* X, double* out,
                       hipStream_t st) {
  const int N = p.n;
  const long NN = (long)N * N;
  if (structured_chain(p)) {
    KronArgs k{};
    k.in = X;
    k.strideIn = NN;
    k.out = out;
    k.strideOut = NN;
    k.s = s;
    k.slice0 = l0;
    k.count = l1 - l0;
    k.step = 1;
    k.scale = 1;
    k.batch = batch;
    return launch_kron(p, k, st);
  }
  // dense products, ping-pong between out and Xb
  GemmArgs g{};
  g.M = N;
  g.N = N;
  g.K = N;
  g.A = p.E;
  g.lda = N;
  g.ldb = N;
  g.strideB = NN;
  g.ldc = N;
  g.strideC = NN;
  g.S = s;
  g.strideS = (long)p.L * N;
  g.consts = p.consts;
  g.alpha = 1.0;
  g.batch = batch;
  const int n = l1 - l0;
  const double* cur = X;
  for (int j = 0; j < n; ++j) {
    double* dst = ((n - 1 - j) % 2 == 0) ? out : p.Xb;
    g.B = cur;
    g.C = dst;
    g.slice = l0 + j;
    SLQ_TRY(launch_gemm(g, false, false, st));
    cur = dst;
  }
  return SLQ_OK;
}

}  // namespace slq

// G(tau_l, 0) = B_l ... B_1 G: the equal-time G of the stabilised chain, then
// the slice products applied to it in blocks of at most n_stab slices.  The
// product multiplies G's columns by up to exp(tau ||K + V||); it is accurate
// while that factor stays far inside the FP64 range relative to the entries
// of G (beta of a few units at the workloads' couplings), which is where
// G(tau, 0) is measured here.
extern "C" int slq_green_displaced(slq_plan* plan, int32_t batch, const int8_t* d_s, int32_t slice, double* d_Gt,
                                   int32_t* d_status, hipStream_t st) {
  if (!plan || !d_s || !d_Gt) {
    set_error("NULL argument");
    return SLQ_ERR_ARG;
  }
  Plan& p = plan->p;
  SLQ_TRY(check_batch(p, batch));
  if (slice < 1 || slice > p.L) {
    set_error("slice must be in [1, L]");
    return SLQ_ERR_ARG;
  }
  if (batch == 0) return SLQ_OK;
  SLQ_HIP(hipSetDevice(p.device));
  const int N = p.n, ns = p.m.n_stab;
  const long NN = (long)N * N;
  int32_t* status = d_status ? d_status : p.status;
  SLQ_TRY(fill_i32(status, batch, 0, st));
  SLQ_TRY(launch_check_spins(p, batch, d_s, status, st));
  SLQ_TRY(run_chain(p, batch, d_s, 0, status, st));
  SLQ_TRY(launch_finish(p, batch, d_Gt, p.dvec, p.sgn_work, status, st));  // G
  for (int l0 = 0; l0 < slice; l0 += ns) {
    const int l1 = std::min(l0 + ns, slice);
    SLQ_TRY(chain_apply(p, batch, d_s, l0, l1, d_Gt, p.Xa, st));         // B(l1, l0) X
    SLQ_TRY(copy_f64(p.Xa, d_Gt, NN * batch, st));
  }
  return SLQ_OK;
}
