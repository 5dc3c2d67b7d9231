// Exact slice products that use the structure of the kinetic factor.
//
// On the periodic lx x ly lattice K is a Kronecker sum (hopping along x plus
// hopping along y, "Basics of DQMC"), so with site i = x + lx y
//     E = exp(-dtau K) = e^{dtau mu} Cx (x) Cy,   (Cx)_{x'x} = Px[(x' - x) mod lx],
// a product of two circulant matrices, and E^{-1} the same with dtau -> -dtau.
// E v for a vector v of N = lx ly entries is lx-point circulant products along
// every x-line followed by ly-point products along every y-line:
// 2N(lx + ly) flops instead of the 2N^2 of a dense product, the same exact
// operator (only the rounding order differs).  This is the role the paper's
// cost count gives to a sparse form of B ("beta N^2" for the whole chain).
//
// A workgroup keeps nb vectors (columns, or rows, of one N x N matrix) in LDS
// and applies a whole block of slices to them, so a block of n_stab slices
// reads and writes each matrix once from HBM.  Each thread holds one lattice
// line in registers; the circulant coefficients are wave-uniform (scalar
// loads from a short window table).
#include <algorithm>
#include <type_traits>

#include "slq_internal.h"

namespace slq {

typedef double d4_t __attribute__((ext_vector_type(4)));

struct KronDev {
  int lx, ly, N, L;
  const double* in;  // null: the identity
  long strideIn;
  double* out;
  long strideOut;
  int rows;  // 0: act on the columns of the matrix, 1: on its rows
  const int8_t* s;
  long strideS;
  int slice0, count, step;
  int scale;  // 0: none, 1: diag(d) before the kinetic factor, 2: after it
  int lognb;  // vectors per workgroup = 1 << lognb
  const double* wx;  // coefficient windows, 2P entries each
  const double* wy;
  const double* consts;  // [0] exp(-dtau xi), [1] exp(+dtau xi)
  int inv;               // 1/d instead of d
  int nvb, batch;        // vector blocks per field, fields
  double* norm2;         // columns mode: squared 2-norms of the output columns, or null
  const int32_t* first_block;  // [batch] or null: fields with block < first_block[b] pass X through
  int block;                   // stabilisation block of this launch
};

// Window w of length 2P for a circulant of period n with first column c:
// C[o][x] = c[(o - x) mod n] = w[x + n - 1 - o] for 0 <= o < n, 0 <= x < P.
__global__ void k_kron_windows(int lx, int ly, int P, const double* __restrict__ tabs,
                               const double* __restrict__ consts, double* __restrict__ w) {
  const int t = threadIdx.x;  // 4 windows x 2P entries
  if (t >= 8 * P) return;
  const int which = t / (2 * P), j = t % (2 * P);
  const bool xdir = (which & 1) == 0, inv = which >= 2;
  const int n = xdir ? lx : ly;
  const double* c = tabs + (inv ? lx + ly : 0) + (xdir ? 0 : lx);
  const double f = xdir ? consts[inv ? 3 : 2] : 1.0;  // e^{+-dtau mu} on the x factor
  const int d = (((n - 1 - j) % n) + n) % n;
  w[t] = f * c[d];
}

// Coefficient windows are read-only for the whole launch: through the constant
// address space the wave-uniform reads become scalar loads.
typedef const __attribute__((address_space(4))) double* cdptr;

// One lattice line (n <= P entries, stride `stride` in LDS) times the circulant
// of window w, in place.  EXACT: n == P, no padding.
template <int P, bool EXACT>
__device__ __forceinline__ void line_product(double* __restrict__ S, int base, int stride, int n, cdptr w,
                                             const double* __restrict__ dl, int dbase, int dstride, int scale) {
  double r[P];
#pragma unroll
  for (int x = 0; x < P; ++x) {
    double v = 0.0;
    if (EXACT || x < n) {
      v = S[base + x * stride];
      if (scale == 1) v *= dl[dbase + x * dstride];
    }
    r[x] = v;
  }
#pragma unroll 2
  for (int o = 0; o < (EXACT ? P : n); ++o) {
    cdptr wo = w + ((EXACT ? P : n) - 1 - o);
    double acc = 0.0;
#pragma unroll
    for (int x = 0; x < P; ++x) acc = fma(wo[x], r[x], acc);
    if (scale == 2) acc *= dl[dbase + o * dstride];
    S[base + o * stride] = acc;
  }
}

// Exact line length P <= 32: both loops unrolled and the circulant read from
// its P/2 + 1 distinct values (its first column is symmetric, c[d] = c[P - d]),
// which stay in scalar registers for the whole launch.
template <int P>
__device__ __forceinline__ void line_product_sym(double* __restrict__ S, int base, int stride,
                                                 const double (&c)[P / 2 + 1], const double* __restrict__ dl,
                                                 int dbase, int dstride, int scale) {
  double r[P];
#pragma unroll
  for (int x = 0; x < P; ++x) {
    double v = S[base + x * stride];
    if (scale == 1) v *= dl[dbase + x * dstride];
    r[x] = v;
  }
  constexpr int OB = P % 4 == 0 ? 4 : (P % 2 == 0 ? 2 : 1);  // independent accumulators
#pragma unroll
  for (int o0 = 0; o0 < P; o0 += OB) {
    double acc[OB];
#pragma unroll
    for (int q = 0; q < OB; ++q) acc[q] = 0.0;
#pragma unroll
    for (int x = 0; x < P; ++x)
#pragma unroll
      for (int q = 0; q < OB; ++q) {
        const int d = ((o0 + q - x) % P + P) % P;
        acc[q] = fma(c[d <= P / 2 ? d : P - d], r[x], acc[q]);
      }
#pragma unroll
    for (int q = 0; q < OB; ++q) {
      double v = acc[q];
      if (scale == 2) v *= dl[dbase + (o0 + q) * dstride];
      S[base + (o0 + q) * stride] = v;
    }
  }
}

// The same with compile-time strides (STRIDE between entries in S, DSTRIDE in
// d_l): every LDS address is a per-thread base plus an instruction offset.
// H lanes share a line: lane h of them computes the outputs o = H k + h.  It
// reads the line rotated by h, r[x] = v[(x + h) mod P]; since the operator is
// circulant, output H k + h of the line is output H k of the rotated one, so
// all H lanes run the same instructions with the same coefficients.  The H
// lanes sit side by side in one wavefront, whose reads of the line all
// complete before its first write, so the in-place update needs no barrier.
template <int P, int STRIDE, int DSTRIDE, int H, int SCALE, class Coef>
__device__ __forceinline__ void line_product_symc(double* __restrict__ S, int base, const Coef& cv,
                                                  const double* __restrict__ dl, int dbase, int h, double f = 1.0) {
  static_assert(P % H == 0, "the lanes of a line split its outputs evenly");
  const int rb = base + h * STRIDE, rdb = dbase + h * DSTRIDE;
  double r[P];
#pragma unroll
  for (int x = 0; x < P; ++x) {
    int o = rb + x * STRIDE, od = rdb + x * DSTRIDE;
    if (x >= P - H + 1 && x + h >= P) {  // wraps round the periodic line
      o -= P * STRIDE;
      od -= P * DSTRIDE;
    }
    double v = S[o];
    if constexpr (SCALE == 1) v *= dl[od];
    r[x] = v;
  }
  constexpr int PO = P / H;  // outputs per lane
  constexpr int OB = PO % 4 == 0 ? 4 : (PO % 5 == 0 ? 5 : (PO % 3 == 0 ? 3 : (PO % 2 == 0 ? 2 : 1)));
#pragma unroll
  for (int k0 = 0; k0 < PO; k0 += OB) {
    double acc[OB];
#pragma unroll
    for (int q = 0; q < OB; ++q) acc[q] = 0.0;
#pragma unroll
    for (int x = 0; x < P; ++x)
#pragma unroll
      for (int q = 0; q < OB; ++q) {
        const int d = ((H * (k0 + q) - x) % P + P) % P;  // coefficient c[d], c symmetric
        acc[q] = fma(cv(d <= P / 2 ? d : P - d), r[x], acc[q]);
      }
#pragma unroll
    for (int q = 0; q < OB; ++q) {
      double v = acc[q];
      if constexpr (SCALE == 2) v *= dl[rdb + H * (k0 + q) * DSTRIDE];
      if constexpr (SCALE == 3) v *= f;
      S[rb + H * (k0 + q) * STRIDE] = v;
    }
  }
}

// Lanes per line of the compile-time path: two wherever the thread count
// allows; four on 48-point lines (2 vectors per workgroup: a 96-register line
// leaves room for three wavefronts per SIMD only when the workgroup has them)
constexpr int kron_lanes_per_line(int P, int nbt) {
  return P == 48 && 4 * P * nbt <= 512 ? 4 : (2 * P * nbt <= (P >= 32 ? 512 : 1024) ? 2 : 1);
}
// and its workgroup size
constexpr int kron_fixed_threads(int P, int nbt) { return (P * nbt * kron_lanes_per_line(P, nbt) + 63) / 64 * 64; }


// NBT > 0: NBT vectors per workgroup and an exact P x P lattice, fixed at
// compile time, so that every LDS address of the line products is a base
// plus an instruction offset (with 8 vectors and P <= 20 at most 72 VGPRs,
// seven wavefronts per SIMD: at 20 x 20 the five workgroups whose blocks fit
// in LDS are then resident together) and every global load of a thread is in flight
// before the first is waited for; NBT = 0: sizes from the arguments.
template <int P, bool EXACT, int NBT>
__global__ __launch_bounds__(P >= 32 ? 512 : 1024) __attribute__((amdgpu_waves_per_eu(NBT == 8 && P <= 20 ? 7 : (P == 48 && NBT ? 3 : 1)))) void k_kron(KronDev a) {
  extern __shared__ double S[];  // [N][nb], then d_l [2][N] (alternating slices)
  const int lin = kron_item((int)blockIdx.x, kron_group(NBT ? NBT : 1 << a.lognb));
  if (lin >= a.nvb * a.batch) return;
  const int lg = NBT ? __builtin_ctz(NBT) : a.lognb, nb = NBT ? NBT : 1 << lg, N = a.N, lx = a.lx, ly = a.ly;
  constexpr int ROWS = P * NBT;  // NBT > 0: stride of lattice rows in S
  const int nS = N * nb;         // doubles of the vector block
  const int tid = threadIdx.x, nt = blockDim.x;  // nt is a multiple of 64, nb <= 32
  const int c = tid & (nb - 1);  // the vector of this thread in loads and stores
  const double dpos = a.consts[a.inv ? 1 : 0], dneg = a.consts[a.inv ? 0 : 1];  // d for s = +1, -1
  // distinct circulant values c[d] = w[P - 1 - d], d = 0..P/2 (exact lines only)
  double cx[P / 2 + 1], cy[P / 2 + 1];
  if constexpr (NBT == 0 && EXACT && P <= 32) {
#pragma unroll
    for (int d = 0; d <= P / 2; ++d) {
      cx[d] = ((cdptr)a.wx)[P - 1 - d];
      cy[d] = ((cdptr)a.wy)[P - 1 - d];
    }
  }
  // compile-time path (square lattice): the x and y lines share one circulant,
  // the y window's (the x window is e^{+-dtau mu} times it), read once into
  // scalar registers; the scalar e^{+-dtau mu} rides on the field factors d_l
  // (or on the x-line outputs when there are none)
  // (up to P = 24: beyond, the registers run short and the values are read
  // from the constant windows as the products go)
  constexpr bool CREG = NBT > 0 && P <= 24;
  double cw[CREG ? P / 2 + 1 : 1];
  double fmu = 1.0;
  if constexpr (CREG) {
#pragma unroll
    for (int d = 0; d <= P / 2; ++d) cw[d] = ((cdptr)a.wy)[P - 1 - d];
    fmu = a.consts[a.inv ? 3 : 2];
  }
  const double dposl = dpos * fmu, dnegl = dneg * fmu;
  const int b = lin / a.nvb;
  // a field whose chain starts at a later block passes X (the identity) through
  const bool idle = a.first_block && a.block < a.first_block[b];
  const int v0 = (lin % a.nvb) * nb;
  const int nv = min(nb, N - v0);
  auto spins = [&](int k) {  // the field of the k-th slice of this launch
    int sl = (a.slice0 + k * a.step) % a.L;
    if (sl < 0) sl += a.L;
    return a.s + (long)b * a.strideS + (long)sl * N;
  };
  // NBT > 0: the thread count and N are compile-time; a thread holds rows
  // (tid / NBT) + q RP, q < NP, of vector c of the block, and the spins of
  // sites tid + q NTF, q < SPT, of the next slice (loaded one slice ahead)
  constexpr int NTF = NBT ? kron_fixed_threads(P, NBT) : 64;
  constexpr int RP = NBT ? NTF / NBT : 1, NP = NBT ? (P * P + RP - 1) / RP : 1;
  constexpr int SPT = NBT ? (P * P + NTF - 1) / NTF : 1;
  int8_t spn[SPT];
  auto prefetch = [&](const int8_t* __restrict__ f) {
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int i = tid + q * NTF;
      spn[q] = i < N ? f[i] : 1;
    }
  };
  if (NBT > 0 && a.scale && !idle) prefetch(spins(0));
  if (!a.rows) {
    if constexpr (NBT > 0) {
      // every load of the thread in flight before the first is stored
      const double* __restrict__ in = a.in ? a.in + (long)b * a.strideIn : nullptr;
      const int j = v0 + c;
      double ent[NP];
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const int i = (tid >> lg) + q * RP;
        ent[q] = 0.0;
        if (i < N && c < nv) ent[q] = in ? in[(long)i * N + j] : (i == j ? 1.0 : 0.0);
      }
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const int i = (tid >> lg) + q * RP;
        if (i < N) S[i * nb + c] = ent[q];
      }
    } else {
      const double* __restrict__ in = a.in ? a.in + (long)b * a.strideIn : nullptr;
      const int j = v0 + c;
      for (int i = tid >> lg; i < N; i += nt >> lg) {
        double v = 0.0;
        if (c < nv) v = in ? in[(long)i * N + j] : (i == j ? 1.0 : 0.0);
        S[i * nb + c] = v;
      }
    }
  } else {
    const double* __restrict__ in = a.in ? a.in + (long)b * a.strideIn : nullptr;
    for (int cc = 0; cc < nb; ++cc) {
      const int j = v0 + cc;
      for (int i = tid; i < N; i += nt) {
        double v = 0.0;
        if (cc < nv) v = in ? in[(long)j * N + i] : (i == j ? 1.0 : 0.0);
        S[i * nb + cc] = v;
      }
    }
  }
  for (int k = 0; k < (idle ? 0 : a.count); ++k) {
    // a second buffer: threads still in the y-lines of slice k - 1 may read the first
    double* dl = S + nS + (k & 1) * N;
    if (a.scale) {
      if constexpr (NBT > 0) {
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
          const int i = tid + q * NTF;
          if (i < N) dl[i] = spn[q] > 0 ? dposl : dnegl;
        }
        if (k + 1 < a.count) prefetch(spins(k + 1));
      } else {
        const int8_t* __restrict__ f = spins(k);
        for (int i = tid; i < N; i += nt) dl[i] = f[i] > 0 ? dpos : dneg;
      }
    }
    __syncthreads();
    if constexpr (NBT > 0) {
      static_assert(EXACT && (P <= 32 || P == 48), "compile-time blocks need an exact lattice of side <= 32 or 48");
      constexpr int H = kron_lanes_per_line(P, NBT);
      const int t = tid / H, h = tid % H;
      const auto creg = [&](int d) { return cw[d]; };
      const auto cwx = [&](int d) { return ((cdptr)a.wx)[P - 1 - d]; };
      const auto cwy = [&](int d) { return ((cdptr)a.wy)[P - 1 - d]; };
      if (t < P * NBT) {  // x-lines
        const int y = t / NBT, cl = t % NBT;
        if constexpr (CREG) {
          if (a.scale == 1)
            line_product_symc<P, NBT, 1, H, 1>(S, y * ROWS + cl, creg, dl, y * P, h);
          else if (a.scale == 2)
            line_product_symc<P, NBT, 1, H, 0>(S, y * ROWS + cl, creg, dl, y * P, h);
          else
            line_product_symc<P, NBT, 1, H, 3>(S, y * ROWS + cl, creg, dl, y * P, h, fmu);
        } else {
          if (a.scale == 1)
            line_product_symc<P, NBT, 1, H, 1>(S, y * ROWS + cl, cwx, dl, y * P, h);
          else
            line_product_symc<P, NBT, 1, H, 0>(S, y * ROWS + cl, cwx, dl, y * P, h);
        }
      }
      __syncthreads();
      if (t < P * NBT) {  // y-lines
        const int x = t / NBT, cl = t % NBT;
        if constexpr (CREG) {
          if (a.scale == 2)
            line_product_symc<P, ROWS, P, H, 2>(S, x * NBT + cl, creg, dl, x, h);
          else
            line_product_symc<P, ROWS, P, H, 0>(S, x * NBT + cl, creg, dl, x, h);
        } else {
          if (a.scale == 2)
            line_product_symc<P, ROWS, P, H, 2>(S, x * NBT + cl, cwy, dl, x, h);
          else
            line_product_symc<P, ROWS, P, H, 0>(S, x * NBT + cl, cwy, dl, x, h);
        }
      }
    } else if constexpr (EXACT && P <= 32) {
      if (tid < ly * nb) {  // x-lines: entries y lx + x, x = 0..lx-1
        const int y = tid >> lg, cl = tid & (nb - 1);
        line_product_sym<P>(S, y * lx * nb + cl, nb, cx, dl, y * lx, 1, a.scale == 1 ? 1 : 0);
      }
      __syncthreads();
      if (tid < lx * nb) {  // y-lines: entries y lx + x, y = 0..ly-1
        const int x = tid >> lg, cl = tid & (nb - 1);
        line_product_sym<P>(S, x * nb + cl, lx * nb, cy, dl, x, lx, a.scale == 2 ? 2 : 0);
      }
    } else {
      if (tid < ly * nb) {  // x-lines: entries y lx + x, x = 0..lx-1
        const int y = tid >> lg, cl = tid & (nb - 1);
        line_product<P, EXACT>(S, y * lx * nb + cl, nb, lx, (cdptr)a.wx, dl, y * lx, 1, a.scale == 1 ? 1 : 0);
      }
      __syncthreads();
      if (tid < lx * nb) {  // y-lines: entries y lx + x, y = 0..ly-1
        const int x = tid >> lg, cl = tid & (nb - 1);
        line_product<P, EXACT>(S, x * nb + cl, lx * nb, ly, (cdptr)a.wy, dl, x, lx, a.scale == 2 ? 2 : 0);
      }
    }
  }
  __syncthreads();
  double* out = a.out + (long)b * a.strideOut;
  if (!a.rows) {
    const int j = v0 + c;
    double ss = 0.0;
    if (c < nv) {
      if constexpr (NBT > 0) {
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          const int i = (tid >> lg) + q * RP;
          if (i < N) {
            const double v = S[i * nb + c];
            out[(long)i * N + j] = v;
            ss += v * v;
          }
        }
      } else {
        for (int i = tid >> lg; i < N; i += nt >> lg) {
          const double v = S[i * nb + c];
          out[(long)i * N + j] = v;
          ss += v * v;
        }
      }
    }
    if (a.norm2) {  // lanes equal mod nb hold parts of one column; then one partial per wave
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1)
        if (o >= nb) ss += __shfl_xor(ss, o, 64);
      double* part = S + nS + 2 * N;  // [waves][nb]
      if ((tid & 63) < nb) part[(tid >> 6) * nb + (tid & 63)] = ss;
      __syncthreads();
      if (tid < nv) {
        double t = 0.0;
        for (int w = 0; w < (nt >> 6); ++w) t += part[w * nb + tid];
        a.norm2[(long)b * N + v0 + tid] = t;
      }
    }
  } else {
    for (int cc = 0; cc < nv; ++cc) {
      const int j = v0 + cc;
      for (int i = tid; i < N; i += nt) out[(long)j * N + i] = S[i * nb + cc];
    }
  }
}

// 48 x 48 lattice, columns, B_l = E diag(d_l), on the matrix cores.  A vector
// of the block is the 48 x 48 grid G[y][x] of its sites (i = x + 48 y), and
// E diag(d) G = e^{dtau mu} Cy (diag(d) G) Cx^T with Cx = Cy = C, the
// 48-point circulant of the y window (on the square lattice the x window is
// e^{+-dtau mu} times it; that factor rides on d).  Wavefront w of the workgroup owns the
// 16-row strip s = w mod 3 of vector w / 3 and computes, with
// v_mfma_f64_16x16x4_f64 (16 x 16 blocks, K = 48 in 12 steps of 4):
//   T^T[:, strip] = G^T C^T[:, strip]   (the y-lines; A from the grid in LDS)
//   G'[strip, :]  = T[strip, :] C^T     (the x-lines; A straight from the
//                                        first product's accumulators)
// The accumulator of block (a, s) of T^T holds, in register r of lane l,
// T[16 s + l % 16][16 a + 4 r + l / 16], which is the A operand of K step
// 4 a + r of the second product, so T never goes through LDS.  The B operands
// are circulant: block (k, b) of C^T depends on (k - 4 b) mod 12 only, so the
// twelve distinct operands stay in registers for the whole launch.
constexpr int KM_P = 48, KM_NB = 4, KM_WAVES = 3 * KM_NB, KM_THREADS = 64 * KM_WAVES;
constexpr int KM_N = KM_P * KM_P;

__global__ __launch_bounds__(KM_THREADS) __attribute__((amdgpu_waves_per_eu(6))) void k_kron_mma48(KronDev a) {
  extern __shared__ double S[];  // [KM_NB][N] grids, then the next slice's spins [N] (bytes), then norm parts
  int8_t* sp = (int8_t*)(S + KM_NB * KM_N);
  double* part = (double*)(sp + KM_N);  // [KM_WAVES][KM_NB]
  const int lin = kron_item((int)blockIdx.x, kron_group(KM_NB));
  if (lin >= a.nvb * a.batch) return;
  const int b = lin / a.nvb, v0 = (lin % a.nvb) * KM_NB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int vw = wave / 3, strip = wave % 3;
  const double fmu = a.consts[a.inv ? 3 : 2];
  const double dpos = a.consts[a.inv ? 1 : 0] * fmu, dneg = a.consts[a.inv ? 0 : 1] * fmu;
  const bool idle = a.first_block && a.block < a.first_block[b];
  auto spins = [&](int k) {
    int sl = (a.slice0 + k * a.step) % a.L;
    if (sl < 0) sl += a.L;
    return a.s + (long)b * a.strideS + (long)sl * KM_N;
  };
  // the twelve B operands: F[q] = C^T[4 k + l / 16][16 b + l % 16] for (k - 4 b) mod 12 = q,
  // i.e. c[(l % 16 - l / 16 - 4 q) mod 48], c[d] = wy[47 - d]
  double F[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) {
    const int d = (((lane & 15) - (lane >> 4) - 4 * q) % KM_P + KM_P) % KM_P;
    F[q] = a.wy[KM_P - 1 - d];
  }
  // the block of vectors, scaled by the first slice's d (sites i, vector c fastest)
  {
    const double* __restrict__ in = a.in ? a.in + (long)b * a.strideIn : nullptr;
    const int8_t* __restrict__ f0 = spins(0);
    const bool sc = !idle && a.count > 0;
    for (int e = tid; e < KM_N * KM_NB; e += KM_THREADS) {
      const int i = e / KM_NB, c = e % KM_NB, j = v0 + c;
      double v = in ? in[(long)i * KM_N + j] : (i == j ? 1.0 : 0.0);
      if (sc) v *= f0[i] > 0 ? dpos : dneg;
      S[c * KM_N + i] = v;
    }
  }
  __syncthreads();
  const double* G = S + vw * KM_N;
  const int rA = lane >> 4, cA = lane & 15;
  for (int k = 0; k < (idle ? 0 : a.count); ++k) {
    const bool more = k + 1 < a.count;
    int8_t nsp[KM_N / KM_THREADS];
    if (more) {
      const int8_t* __restrict__ f = spins(k + 1);
#pragma unroll
      for (int q = 0; q < KM_N / KM_THREADS; ++q) nsp[q] = f[tid + q * KM_THREADS];
    }
    // T^T blocks (a, strip), a = 0..2: A = G^T block (a, kk): G[4 kk + l / 16][16 a + l % 16]
    d4_t t[3];
#pragma unroll
    for (int aa = 0; aa < 3; ++aa) t[aa] = d4_t{0.0, 0.0, 0.0, 0.0};
    auto ylines = [&](auto st_) {  // the strip as a compile-time constant: F indexed statically
      constexpr int st = decltype(st_)::value;
#pragma unroll
      for (int kk = 0; kk < 12; ++kk) {
        const double* row = G + (4 * kk + rA) * KM_P + cA;
        const int q = ((kk - 4 * st) % 12 + 12) % 12;
#pragma unroll
        for (int aa = 0; aa < 3; ++aa) t[aa] = __builtin_amdgcn_mfma_f64_16x16x4f64(row[16 * aa], F[q], t[aa], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);  // K step by K step: three operands in registers at a time
      }
    };
    if (strip == 0)
      ylines(std::integral_constant<int, 0>{});
    else if (strip == 1)
      ylines(std::integral_constant<int, 1>{});
    else
      ylines(std::integral_constant<int, 2>{});
    if (more) {
#pragma unroll
      for (int q = 0; q < KM_N / KM_THREADS; ++q) sp[tid + q * KM_THREADS] = nsp[q];
    }
    __syncthreads();  // every wave has read the grids; the next spins are in LDS
    // G' blocks (strip, bj): A operand of K step kk = 4 aa + r is register r of t[aa]
    double* Gw = S + vw * KM_N;
#pragma unroll
    for (int bj = 0; bj < 3; ++bj) {
      d4_t g = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 12; ++kk) {
        const int q = ((kk - 4 * bj) % 12 + 12) % 12;
        g = __builtin_amdgcn_mfma_f64_16x16x4f64(t[kk >> 2][kk & 3], F[q], g, 0, 0, 0);
      }
      // register r of lane l: G'[16 strip + 4 r + l / 16][16 bj + l % 16], times the next slice's d
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = (16 * strip + 4 * r + rA) * KM_P + 16 * bj + cA;
        double v = g[r];
        if (more) v *= sp[i] > 0 ? dpos : dneg;
        Gw[i] = v;
      }
      __builtin_amdgcn_sched_barrier(0);  // one output block's accumulators live at a time
    }
    __syncthreads();
  }
  // out, and the squared norms of the output columns
  double* __restrict__ out = a.out + (long)b * a.strideOut;
  const int c = tid % KM_NB;
  double ss = 0.0;
  for (int i = tid / KM_NB; i < KM_N; i += KM_THREADS / KM_NB) {
    const double v = S[c * KM_N + i];
    out[(long)i * KM_N + v0 + c] = v;
    ss += v * v;
  }
  if (a.norm2) {  // lanes equal mod KM_NB hold parts of one column
#pragma unroll
    for (int o = 32; o >= KM_NB; o >>= 1) ss += __shfl_xor(ss, o, 64);
    if (lane < KM_NB) part[wave * KM_NB + lane] = ss;
    __syncthreads();
    if (tid < KM_NB) {
      double tt = 0.0;
      for (int w = 0; w < KM_WAVES; ++w) tt += part[w * KM_NB + tid];
      a.norm2[(long)b * KM_N + v0 + tid] = tt;
    }
  }
}

static const int kKronSizes[] = {4, 8, 12, 16, 20, 24, 32, 40, 48, 64};

int kron_line_size(int lx, int ly) {
  const int m = std::max(lx, ly);
  for (int P : kKronSizes)
    if (P >= m) return P;
  return 0;
}

int launch_kron_windows(Plan& p, hipStream_t st) {
  if (p.kron_P == 0) return SLQ_OK;
  k_kron_windows<<<1, 8 * p.kron_P, 0, st>>>(p.m.lx, p.m.ly, p.kron_P, p.tabs, p.consts, p.kron_w);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

static int kron_max_threads(int P) { return P >= 32 ? 512 : 1024; }

static bool kron_fixed(const Plan& p, int nb) {
  if (p.m.lx != p.kron_P || p.m.ly != p.kron_P) return false;
  return (p.kron_P <= 32 && (nb == 8 || nb == 16)) || (p.kron_P == 48 && (nb == 2 || nb == 4));
}
// threads of a workgroup: one per line and vector, or H per line on the fixed path
static int kron_threads(const Plan& p, int nb) {
  const int m = std::max(p.m.lx, p.m.ly);
  return kron_fixed(p, nb) ? kron_fixed_threads(p.kron_P, nb) : (m * nb + 63) / 64 * 64;
}
// LDS: the block of vectors, two d_l rows, one partial norm per wave and vector
static size_t kron_lds(const Plan& p, int nb) {
  const int waves = kron_threads(p, nb) / 64;
  return ((size_t)p.n * (nb + 2) + (size_t)waves * nb) * sizeof(double);
}

int kron_default_nb(const Plan& p) {
  if (p.cb) return cb_default_nb(p);
  const int m = std::max(p.m.lx, p.m.ly);
  for (int nb = 32; nb > 1; nb /= 2)
    if (kron_lds(p, nb) <= 80 * 1024 && m * nb <= kron_max_threads(p.kron_P)) return nb;
  return 1;
}

template <int P>
static void launch_p(const KronDev& d, bool exact, int nb, bool fixed, dim3 grid, int threads, size_t lds,
                     hipStream_t st) {
  if constexpr (P == 48) {
    if (fixed && nb == 2) {
      allow_max_lds((const void*)k_kron<P, true, 2>);
      k_kron<P, true, 2><<<grid, threads, lds, st>>>(d);
      return;
    }
    if (fixed && nb == 4) {
      allow_max_lds((const void*)k_kron<P, true, 4>);
      k_kron<P, true, 4><<<grid, threads, lds, st>>>(d);
      return;
    }
  }
  if constexpr (P <= 32) {
    if (fixed && nb == 8) {
      allow_max_lds((const void*)k_kron<P, true, 8>);
      k_kron<P, true, 8><<<grid, threads, lds, st>>>(d);
      return;
    }
    if (fixed && nb == 16) {
      allow_max_lds((const void*)k_kron<P, true, 16>);
      k_kron<P, true, 16><<<grid, threads, lds, st>>>(d);
      return;
    }
  }
  if (exact) {
    allow_max_lds((const void*)k_kron<P, true, 0>);
    k_kron<P, true, 0><<<grid, threads, lds, st>>>(d);
  } else {
    allow_max_lds((const void*)k_kron<P, false, 0>);
    k_kron<P, false, 0><<<grid, threads, lds, st>>>(d);
  }
}

bool kron_width_ok(const Plan& p, int nb) {
  if (p.cb) return cb_width_ok(p, nb);
  const int m = std::max(p.m.lx, p.m.ly);
  return nb >= 1 && nb <= 32 && (nb & (nb - 1)) == 0 && m * nb <= kron_max_threads(p.kron_P) &&
         kron_lds(p, nb) <= 160 * 1024;
}

int launch_kron(Plan& p, const KronArgs& a, hipStream_t st) {
  if (p.cb) return launch_cb(p, a, st);
  if (a.batch <= 0 || a.count <= 0) return SLQ_OK;
  if (p.kron_P == 0) {
    set_error("structured slice products need lx, ly <= 64");
    return SLQ_ERR_ARG;
  }
  const int nb = a.nb > 0 ? a.nb : (p.kron_nb > 0 ? p.kron_nb : kron_default_nb(p));
  const bool fixed = kron_fixed(p, nb);
  const size_t lds = kron_lds(p, nb);
  if (!kron_width_ok(p, nb)) {
    set_error("structured slice product: vectors per workgroup must be a power of two <= 32 that fits");
    return SLQ_ERR_ARG;
  }
  int lognb = 0;
  while ((1 << lognb) < nb) ++lognb;
  KronDev d;
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
  d.lognb = lognb;
  const int P = p.kron_P;
  d.wx = p.kron_w + (a.inv ? 4 * P : 0);
  d.wy = d.wx + 2 * P;
  d.consts = p.consts;
  d.inv = a.inv;
  const int threads = kron_threads(p, nb);
  const bool exact = p.m.lx == P && p.m.ly == P;
  d.norm2 = a.rows ? nullptr : a.norm2;
  d.nvb = (p.n + nb - 1) / nb;
  d.batch = a.batch;
  d.first_block = a.first_block;
  d.block = a.block;
  if (P == KM_P && exact && !a.rows && a.scale == 1) {
    // the matrix-core path of the 48 x 48 lattice (its own width of 4 vectors)
    d.nvb = KM_N / KM_NB;
    d.lognb = 2;
    const long gm = 8L * kron_group(KM_NB);
    const size_t lm = sizeof(double) * KM_NB * KM_N + KM_N + sizeof(double) * KM_WAVES * KM_NB;
    allow_max_lds((const void*)k_kron_mma48);
    k_kron_mma48<<<dim3((unsigned)(((long)d.nvb * a.batch + gm - 1) / gm * gm)), KM_THREADS, lm, st>>>(d);
    SLQ_LAUNCHED();
    return SLQ_OK;
  }
  const long gq = 8L * kron_group(nb);
  dim3 grid((unsigned)(((long)d.nvb * a.batch + gq - 1) / gq * gq));
  switch (P) {
    case 4: launch_p<4>(d, exact, nb, fixed, grid, threads, lds, st); break;
    case 8: launch_p<8>(d, exact, nb, fixed, grid, threads, lds, st); break;
    case 12: launch_p<12>(d, exact, nb, fixed, grid, threads, lds, st); break;
    case 16: launch_p<16>(d, exact, nb, fixed, grid, threads, lds, st); break;
    case 20: launch_p<20>(d, exact, nb, fixed, grid, threads, lds, st); break;
    case 24: launch_p<24>(d, exact, nb, fixed, grid, threads, lds, st); break;
    case 32: launch_p<32>(d, exact, nb, fixed, grid, threads, lds, st); break;
    case 40: launch_p<40>(d, exact, nb, fixed, grid, threads, lds, st); break;
    case 48: launch_p<48>(d, exact, nb, fixed, grid, threads, lds, st); break;
    default: launch_p<64>(d, exact, nb, fixed, grid, threads, lds, st); break;
  }
  SLQ_LAUNCHED();
  return SLQ_OK;
}

// Time every admissible number of vectors per workgroup for one n_stab block
// on `batch` fields of the plan's workspace (fields of +1 spins written into
// s_work) and keep the fastest in the plan.  Synchronous on st.
int tune_kron(Plan& p, int batch, hipStream_t st, float* best_ms_out) {
  if (!has_structured(p)) return SLQ_OK;
  const int N = p.n;
  int rc = fill_i32((int32_t*)p.s_work, (long)batch * p.L * N / 4, 0x01010101, st);
  if (rc != SLQ_OK) return rc;
  // timed as in a chain block: read a product, write a product and its column norms
  KronArgs k{};
  k.in = nullptr;
  k.out = p.Xb;
  k.strideOut = (long)N * N;
  k.s = p.s_work;
  k.slice0 = 0;
  k.count = std::min(p.m.n_stab, p.L);
  k.step = 1;
  k.scale = 1;
  k.batch = batch;
  if ((rc = launch_kron(p, k, st)) != SLQ_OK) return rc;
  k.in = p.Xb;
  k.strideIn = (long)N * N;
  k.out = p.Xa;
  k.norm2 = p.xnorm2;
  hipEvent_t e0, e1;
  SLQ_HIP(hipEventCreate(&e0));
  SLQ_HIP(hipEventCreate(&e1));
  int best = 0;
  float best_ms = 1e30f;
  for (int nb = 2; nb <= 32 && rc == SLQ_OK; nb *= 2) {
    k.nb = nb;
    if (launch_kron(p, k, st) != SLQ_OK) continue;  // not admissible for this lattice
    if (hipEventRecord(e0, st) != hipSuccess) rc = SLQ_ERR_DEVICE;
    for (int r = 0; r < 3 && rc == SLQ_OK; ++r) rc = launch_kron(p, k, st);
    float ms = 0.f;
    if (rc == SLQ_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = SLQ_ERR_DEVICE;
    if (rc == SLQ_OK && ms < best_ms) {
      best_ms = ms;
      best = nb;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != SLQ_OK) {
    set_error("timing of the structured chain product failed");
    return rc;
  }
  if (best == 0) {
    set_error("no admissible vector block for the structured chain product");
    return SLQ_ERR_ARG;
  }
  p.kron_nb = best;
  if (best_ms_out) *best_ms_out = best_ms / 3;
  return SLQ_OK;
}

}  // namespace slq
