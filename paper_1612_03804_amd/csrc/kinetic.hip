// Kinetic propagators E = exp(-dtau K) and E^{-1} = exp(+dtau K).
//
// K (hopping -t on nearest-neighbour bonds of the periodic lx x ly lattice,
// -mu on the diagonal; "Basics of DQMC": the kinetic factor of B^tau) is
// diagonal in lattice momentum with eps_k = -2t(cos kx + cos ky) - mu, so
//   E[i][j] = e^{dtau mu} * Px[(x_i - x_j) mod lx] * Py[(y_i - y_j) mod ly],
//   Px[d] = (1/lx) sum_n exp(2 t dtau cos(2 pi n / lx)) cos(2 pi n d / lx),
// and E^{-1} the same with dtau -> -dtau.  Built on the device once per plan.
#include "slq_internal.h"

namespace slq {

// tabs layout: [Px(lx) | Py(ly) | Pxinv(lx) | Pyinv(ly)]; consts: see Plan.
__global__ void k_kinetic_tables(int lx, int ly, double t, double mu, double dtau, double xi, double* tabs,
                                 double* consts) {
  const int tid = threadIdx.x + blockIdx.x * blockDim.x;
  const int total = 2 * (lx + ly);
  if (tid < total) {
    const int half = lx + ly;
    const double sgn = tid < half ? 1.0 : -1.0;  // +: E, -: E^{-1}
    int idx = tid % half;
    int len = lx, d = idx;
    if (idx >= lx) {
      len = ly;
      d = idx - lx;
    }
    double acc = 0.0;
    for (int n = 0; n < len; ++n) {
      const double ek = exp(sgn * 2.0 * t * dtau * cospi(2.0 * (double)n / (double)len));
      acc += ek * cospi(2.0 * (double)((long)n * d % len) / (double)len);
    }
    tabs[tid] = acc / (double)len;
  }
  if (tid == 0) {
    consts[0] = exp(-dtau * xi);
    consts[1] = exp(dtau * xi);
    consts[2] = exp(dtau * mu);
    consts[3] = exp(-dtau * mu);
  }
}

__global__ void k_kinetic_fill(int lx, int ly, const double* __restrict__ tabs, const double* __restrict__ consts,
                               double* __restrict__ E, double* __restrict__ Einv) {
  const int n = lx * ly;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx % n);
  const int dx = ((i % lx) - (j % lx) + lx) % lx;
  const int dy = ((i / lx) - (j / lx) + ly) % ly;
  const double* px = tabs;
  const double* py = tabs + lx;
  const double* pxi = tabs + lx + ly;
  const double* pyi = tabs + 2 * lx + ly;
  E[idx] = consts[2] * px[dx] * py[dy];
  Einv[idx] = consts[3] * pxi[dx] * pyi[dy];
}

int launch_kinetic(Plan& p, hipStream_t st) {
  const slq_model& m = p.m;
  const int total = 2 * (m.lx + m.ly);
  k_kinetic_tables<<<(total + 255) / 256, 256, 0, st>>>(m.lx, m.ly, m.t, m.mu, m.dtau, m.xi, p.tabs, p.consts);
  SLQ_LAUNCHED();
  const long nn = (long)p.n * p.n;
  k_kinetic_fill<<<(unsigned)((nn + 255) / 256), 256, 0, st>>>(m.lx, m.ly, p.tabs, p.consts, p.E, p.Einv);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

}  // namespace slq
