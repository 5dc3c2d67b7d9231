// Checkerboard slice products (SLQ_PREC_CHECKERBOARD).
//
// The cost count of "Formalism of SLDQMC" (beta N^2 for the chain of a
// cumulative update) presumes slice matrices that factor into sparse pieces.
// On an lx x ly torus with even sides the nearest-neighbour bonds fall into
// four groups of disjoint bonds: x bonds leaving an even x (A) or an odd x
// (B), y bonds leaving an even y (C) or an odd y (D).  exp(-dtau K_g) of one
// group is a 2 x 2 rotation [[cosh, sinh], [sinh, cosh]](dtau t) on each of
// its bonds, and the symmetric split
//     E_cb = e^{dtau mu} A' B' C' D C' B' A'   (X' = the half-step factor)
// replaces E = exp(-dtau K) (a discretisation error of the same order as
// the Trotter error of the slices; E_cb^{-1} takes dtau -> -dtau).  Applying
// it to a vector costs 22 N flops (seven bond groups of N/2 rotations
// of 6 flops, and d_l) instead of the 2 N (lx + ly) of the exact
// circulant lines.
//
// A workgroup applies a block of slices to nb vectors (columns, or rows, of
// one N x N matrix).  A thread holds, in registers, the P x P sites of a
// plaquette (x0, y0 multiples of P) of one vector: the A and C bonds,
// and the B and D bonds inside a plaquette, are register-local; only the B
// bond across the right edge and the D bond across the lower edge need the
// neighbouring plaquette, and both threads of such a bond evaluate it from
// the two edge values exchanged through LDS (three exchanges per slice, two
// alternating LDS areas, one barrier each).  HBM sees each matrix once per
// block: read, then written with its column norms.
#include <algorithm>
#include <cmath>

#include "slq_internal.h"

namespace slq {

struct CbDev {
  int lx, ly, N, L;
  const double* in;  // null: the identity
  long strideIn;
  double* out;
  long strideOut;
  int rows;  // 0: act on the columns, 1: on the rows
  const int8_t* s;
  long strideS;
  int slice0, count, step;
  int scale;               // 0: E_cb only, 1: E_cb diag(d), 2: diag(d) E_cb
  double ch, sh, cf, sf;   // cosh, sinh of dtau t / 2 and of dtau t (sinh negated for the inverse)
  double emu;              // e^{+-dtau mu}
  double dpos, dneg;       // d_l for s = +1, -1 (reciprocals for the inverse)
  int nvb, batch;
  int npx, npy;            // plaquettes along x and y
  int s_words;             // P = 4 and 4-byte aligned fields: a plaquette row's spins as one word
  double* norm2;           // columns: squared 2-norms of the output columns, or null
  const int32_t* first_block;
  int block;
};

__device__ __forceinline__ void cb_rot(double& u, double& w, double c, double s) {
  const double a = u, b = w;
  u = c * a + s * b;
  w = s * a + c * b;
}

// Doubles of one LDS exchange area: per plaquette two edges of P sites, nb vectors.
__host__ __device__ inline int cb_area(int N, int P, int nb) { return 2 * (N / P) * nb; }

// P x P plaquettes (P = 4 when both sides are multiples of 4, else 2), QP of
// them per thread (the launcher uses one), NB vectors per workgroup, all
// compile-time so that every register index and every LDS offset of an edge
// is a constant.
template <int P, int QP, int NB>
__global__ __launch_bounds__(QP >= 2 ? 512 : 1024) void k_cb(CbDev a) {
  extern __shared__ double S[];  // two exchange areas [npl][2 edges][P][NB], then one partial norm per thread
  constexpr int PS = P * P;
  const int lin = kron_item((int)blockIdx.x, kron_group(NB));
  if (lin >= a.nvb * a.batch) return;  // uniform over the workgroup
  const int N = a.N, lx = a.lx, npx = a.npx, npy = a.npy, npl = npx * npy;
  const int tid = threadIdx.x, nt = blockDim.x, c = tid % NB, slot = tid / NB, slots = nt / NB;
  const int b = lin / a.nvb, v0 = (lin % a.nvb) * NB, j = v0 + c;
  const bool live = j < N;
  const bool idle = a.first_block && a.block < a.first_block[b];
  const int area = cb_area(N, P, NB);
  double* red = S + 2 * area;

  // per plaquette: its first site and the LDS offsets of its own edges and of
  // the edges its four neighbours write
  bool ok[QP];
  int i0[QP], own[QP], xr[QP], xl[QP], yd[QP], yu[QP];
#pragma unroll
  for (int q = 0; q < QP; ++q) {
    const int p = slot + q * slots;
    ok[q] = p < npl;
    const int px = ok[q] ? p % npx : 0, py = ok[q] ? p / npx : 0;
    i0[q] = px * P + lx * py * P;
    const int pr = (px + 1 == npx ? 0 : px + 1) + npx * py;
    const int pl = (px == 0 ? npx - 1 : px - 1) + npx * py;
    const int pd = px + npx * (py + 1 == npy ? 0 : py + 1);
    const int pu = px + npx * (py == 0 ? npy - 1 : py - 1);
    own[q] = (px + npx * py) * 2 * P * NB + c;
    xr[q] = pr * 2 * P * NB + c;          // right neighbour's first edge (its left column)
    xl[q] = (pl * 2 + 1) * P * NB + c;    // left neighbour's second edge (its right column)
    yd[q] = pd * 2 * P * NB + c;          // lower neighbour's top row
    yu[q] = (pu * 2 + 1) * P * NB + c;    // upper neighbour's bottom row
  }

  double v[QP][PS];
  {
    const double* __restrict__ in = a.in ? a.in + (long)b * a.strideIn : nullptr;
#pragma unroll
    for (int q = 0; q < QP; ++q)
#pragma unroll
      for (int e = 0; e < PS; ++e) {
        const int i = i0[q] + e % P + lx * (e / P);
        double x = 0.0;
        if (ok[q] && live) {
          if (in)
            x = a.rows ? in[(long)j * N + i] : in[(long)i * N + j];
          else
            x = i == j ? 1.0 : 0.0;
        }
        v[q][e] = x;
      }
  }

  int xc = 0;  // exchange counter: the LDS area in use alternates
  // B bonds (x0 + P - 1, x0 + P) across the right edge of every plaquette:
  // edge 0 = left column, edge 1 = right column
  auto exchange_x = [&](double cc, double ss) {
    double* E = S + (xc & 1) * area;
    ++xc;
#pragma unroll
    for (int q = 0; q < QP; ++q)
      if (ok[q]) {
#pragma unroll
        for (int d = 0; d < P; ++d) {
          E[own[q] + d * NB] = v[q][d * P];
          E[own[q] + (P + d) * NB] = v[q][d * P + P - 1];
        }
      }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QP; ++q)
      if (ok[q]) {
#pragma unroll
        for (int d = 0; d < P; ++d) {
          const double r = E[xr[q] + d * NB], l = E[xl[q] + d * NB];
          double& vl = v[q][d * P];
          double& vr = v[q][d * P + P - 1];
          const double nr = cc * vr + ss * r;
          const double nl = ss * l + cc * vl;
          vr = nr;
          vl = nl;
        }
      }
  };
  // D bonds (y0 + P - 1, y0 + P) across the lower edge: edge 0 = top row, edge 1 = bottom row
  auto exchange_y = [&](double cc, double ss) {
    double* E = S + (xc & 1) * area;
    ++xc;
#pragma unroll
    for (int q = 0; q < QP; ++q)
      if (ok[q]) {
#pragma unroll
        for (int d = 0; d < P; ++d) {
          E[own[q] + d * NB] = v[q][d];
          E[own[q] + (P + d) * NB] = v[q][(P - 1) * P + d];
        }
      }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QP; ++q)
      if (ok[q]) {
#pragma unroll
        for (int d = 0; d < P; ++d) {
          const double dn = E[yd[q] + d * NB], up = E[yu[q] + d * NB];
          double& vt = v[q][d];
          double& vb = v[q][(P - 1) * P + d];
          const double nb = cc * vb + ss * dn;
          const double nt = ss * up + cc * vt;
          vb = nb;
          vt = nt;
        }
      }
  };
  auto local_x = [&](int start, double cc, double ss) {  // bonds (x0 + dx, x0 + dx + 1), dx = start, start + 2, ...
#pragma unroll
    for (int q = 0; q < QP; ++q)
#pragma unroll
      for (int dy = 0; dy < P; ++dy)
#pragma unroll
        for (int dx = start; dx + 1 < P; dx += 2) cb_rot(v[q][dy * P + dx], v[q][dy * P + dx + 1], cc, ss);
  };
  auto local_y = [&](int start, double cc, double ss) {
#pragma unroll
    for (int q = 0; q < QP; ++q)
#pragma unroll
      for (int dy = start; dy + 1 < P; dy += 2)
#pragma unroll
        for (int dx = 0; dx < P; ++dx) cb_rot(v[q][dy * P + dx], v[q][(dy + 1) * P + dx], cc, ss);
  };
  const double dpos = a.dpos * a.emu, dneg = a.dneg * a.emu;  // e^{+-dtau mu} rides on d_l
  auto scale_by = [&](int k) {  // v_i *= d_l(i) e^{dtau mu} for the k-th slice of the launch
    int sl = (a.slice0 + k * a.step) % a.L;
    if (sl < 0) sl += a.L;
    const int8_t* __restrict__ f = a.s + (long)b * a.strideS + (long)sl * N;
#pragma unroll
    for (int q = 0; q < QP; ++q)
#pragma unroll
      for (int dy = 0; dy < P; ++dy) {
        const int8_t* __restrict__ row = f + (ok[q] ? i0[q] + lx * dy : 0);
        if (P == 4 && a.s_words) {
          const unsigned w = *(const unsigned*)row;
#pragma unroll
          for (int dx = 0; dx < P; ++dx) v[q][dy * P + dx] *= (w >> (8 * dx + 7)) & 1u ? dneg : dpos;
        } else {
#pragma unroll
          for (int dx = 0; dx < P; ++dx) v[q][dy * P + dx] *= row[dx] > 0 ? dpos : dneg;
        }
      }
  };

  for (int k = 0; k < (idle ? 0 : a.count); ++k) {
    if (a.scale == 1) scale_by(k);
    local_x(0, a.ch, a.sh);  // A'
    local_x(1, a.ch, a.sh);  // B' inside the plaquettes
    exchange_x(a.ch, a.sh);  //    and across their right edges
    local_y(0, a.ch, a.sh);  // C'
    local_y(1, a.cf, a.sf);  // D
    exchange_y(a.cf, a.sf);
    local_y(0, a.ch, a.sh);  // C'
    local_x(1, a.ch, a.sh);  // B'
    exchange_x(a.ch, a.sh);
    local_x(0, a.ch, a.sh);  // A'
    if (a.scale == 2) {
      scale_by(k);
    } else if (a.scale == 0) {
#pragma unroll
      for (int q = 0; q < QP; ++q)
#pragma unroll
        for (int e = 0; e < PS; ++e) v[q][e] *= a.emu;
    }
  }

  double part = 0.0;
  {
    double* __restrict__ out = a.out + (long)b * a.strideOut;
#pragma unroll
    for (int q = 0; q < QP; ++q)
#pragma unroll
      for (int e = 0; e < PS; ++e) {
        const int i = i0[q] + e % P + lx * (e / P);
        if (ok[q] && live) {
          if (a.rows)
            out[(long)j * N + i] = v[q][e];
          else
            out[(long)i * N + j] = v[q][e];
          part += v[q][e] * v[q][e];
        }
      }
  }
  if (a.norm2 && !a.rows) {
    red[tid] = part;
    __syncthreads();
    if (tid < NB && v0 + tid < N) {
      double t = 0.0;
      for (int r = tid; r < nt; r += NB) t += red[r];
      a.norm2[(long)b * N + v0 + tid] = t;
    }
  }
}

static int cb_side(const Plan& p) { return p.m.lx % 4 == 0 && p.m.ly % 4 == 0 ? 4 : 2; }

// Threads of a workgroup for nb vectors, one plaquette of one vector each,
// or 0 when they exceed 1024 (a second plaquette per thread would halve the
// threads but not the work per CU: the widths that need it are not admitted).
static int cb_threads(const Plan& p, int nb) {
  const int P = cb_side(p), npl = p.n / (P * P);
  const int nt = (npl * nb + 63) / 64 * 64;
  return nt <= 1024 ? nt : 0;
}

static size_t cb_lds(const Plan& p, int nb) {
  const int nt = cb_threads(p, nb);
  if (!nt) return SIZE_MAX;
  return ((size_t)2 * cb_area(p.n, cb_side(p), nb) + nt) * sizeof(double);
}

bool cb_width_ok(const Plan& p, int nb) {
  return nb >= 1 && nb <= 16 && (nb & (nb - 1)) == 0 && cb_threads(p, nb) > 0 && cb_lds(p, nb) <= 160 * 1024;
}

int cb_default_nb(const Plan& p) {
  for (int nb = 8; nb > 1; nb /= 2)
    if (cb_width_ok(p, nb) && cb_lds(p, nb) <= 80 * 1024) return nb;
  return 1;
}

template <int P>
static void launch_p(const CbDev& d, int nb, dim3 grid, int threads, size_t lds, hipStream_t st) {
  constexpr int QP = 1;
  switch (nb) {
#define SLQ_CB_CASE(NB)                                    \
  case NB:                                                 \
    allow_max_lds((const void*)k_cb<P, QP, NB>);           \
    k_cb<P, QP, NB><<<grid, threads, lds, st>>>(d);        \
    break;
    SLQ_CB_CASE(1)
    SLQ_CB_CASE(2)
    SLQ_CB_CASE(4)
    SLQ_CB_CASE(8)
    SLQ_CB_CASE(16)
#undef SLQ_CB_CASE
  }
}

int launch_cb(Plan& p, const KronArgs& a, hipStream_t st) {
  if (a.batch <= 0 || a.count <= 0) return SLQ_OK;
  const int nb = a.nb > 0 ? a.nb : (p.kron_nb > 0 ? p.kron_nb : cb_default_nb(p));
  if (!cb_width_ok(p, nb)) {
    set_error("checkerboard slice product: vectors per workgroup must be a power of two <= 16 that fits");
    return SLQ_ERR_ARG;
  }
  const int threads = cb_threads(p, nb);
  const int P = cb_side(p);
  CbDev d;
  d.lx = p.m.lx;
  d.ly = p.m.ly;
  d.N = p.n;
  d.L = p.L;
  d.in = a.in;
  d.strideIn = a.strideIn;
  d.out = a.out;
  d.strideOut = a.strideOut;
  d.rows = a.rows;
  d.s = a.s;
  d.strideS = (long)p.L * p.n;
  d.slice0 = a.slice0;
  d.count = a.count;
  d.step = a.step;
  d.scale = a.scale;
  const double sg = a.inv ? -1.0 : 1.0, h = p.m.dtau * p.m.t;
  d.ch = std::cosh(0.5 * h);
  d.sh = sg * std::sinh(0.5 * h);
  d.cf = std::cosh(h);
  d.sf = sg * std::sinh(h);
  d.emu = std::exp(sg * p.m.dtau * p.m.mu);
  d.dpos = std::exp(-sg * p.m.dtau * p.m.xi);
  d.dneg = std::exp(sg * p.m.dtau * p.m.xi);
  d.nvb = (p.n + nb - 1) / nb;
  d.batch = a.batch;
  d.npx = p.m.lx / P;
  d.npy = p.m.ly / P;
  // row starts are multiples of 4 when P = 4 (lx, N and L N are), so the words
  // are aligned when the field array is
  d.s_words = P == 4 && a.s && ((uintptr_t)a.s % 4 == 0);
  d.norm2 = a.rows ? nullptr : a.norm2;
  d.first_block = a.first_block;
  d.block = a.block;
  const size_t lds = cb_lds(p, nb);
  const long gq = 8L * kron_group(nb);
  dim3 grid((unsigned)(((long)d.nvb * a.batch + gq - 1) / gq * gq));
  if (P == 4)
    launch_p<4>(d, nb, grid, threads, lds, st);
  else
    launch_p<2>(d, nb, grid, threads, lds, st);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

// E_cb and E_cb^{-1} as dense matrices (the operator applied to the identity),
// for the products that use a dense kinetic factor.
int launch_cb_dense(Plan& p, hipStream_t st) {
  KronArgs k{};
  k.in = nullptr;
  k.strideOut = (long)p.n * p.n;
  k.count = 1;
  k.step = 1;
  k.scale = 0;
  k.batch = 1;
  k.out = p.E;
  k.inv = 0;
  SLQ_TRY(launch_cb(p, k, st));
  k.out = p.Einv;
  k.inv = 1;
  return launch_cb(p, k, st);
}

}  // namespace slq
