// C ABI of libslq: plans, argument checks and the orchestration of the
// stabilised chain (every arithmetic step runs in the kernels of this library).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "slq_internal.h"

namespace slq {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

static int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

__global__ void k_fill_f64(double* x, long n, double v) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) x[i] = v;
}
__global__ void k_fill_i32(int32_t* x, long n, int32_t v) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) x[i] = v;
}
__global__ void k_fill_i64(int64_t* x, long n, int64_t v) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) x[i] = v;
}
__global__ void k_copy_f64(const double* __restrict__ a, double* __restrict__ b, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) b[i] = a[i];
}
__global__ void k_copy_i8(const int8_t* __restrict__ a, int8_t* __restrict__ b, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) b[i] = a[i];
}

// M[b] = sum of the spins of field b (fixed-order integer reduction).
__global__ __launch_bounds__(256) void k_magnetization(long per, const int8_t* __restrict__ s, int64_t* M) {
  __shared__ long long red[4];
  const int8_t* sb = s + (long)blockIdx.x * per;
  long long acc = 0;
  for (long i = threadIdx.x; i < per; i += 256) acc += sb[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) M[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

static unsigned grid_for(long n) { return (unsigned)std::max<long>(1, std::min<long>((n + 255) / 256, 2048)); }

int fill_f64(double* x, long n, double v, hipStream_t st) {
  if (n <= 0) return SLQ_OK;
  k_fill_f64<<<grid_for(n), 256, 0, st>>>(x, n, v);
  SLQ_LAUNCHED();
  return SLQ_OK;
}
int fill_i32(int32_t* x, long n, int32_t v, hipStream_t st) {
  if (n <= 0) return SLQ_OK;
  k_fill_i32<<<grid_for(n), 256, 0, st>>>(x, n, v);
  SLQ_LAUNCHED();
  return SLQ_OK;
}
int fill_i64(int64_t* x, long n, int64_t v, hipStream_t st) {
  if (n <= 0) return SLQ_OK;
  k_fill_i64<<<grid_for(n), 256, 0, st>>>(x, n, v);
  SLQ_LAUNCHED();
  return SLQ_OK;
}
int copy_f64(const double* a, double* b, long n, hipStream_t st) {
  if (n <= 0) return SLQ_OK;
  k_copy_f64<<<grid_for(n), 256, 0, st>>>(a, b, n);
  SLQ_LAUNCHED();
  return SLQ_OK;
}
int copy_i8(const int8_t* a, int8_t* b, long n, hipStream_t st) {
  if (n <= 0) return SLQ_OK;
  k_copy_i8<<<grid_for(n), 256, 0, st>>>(a, b, n);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

static int check_model(const slq_model* m) {
  if (!m) return fail(SLQ_ERR_ARG, "model is NULL");
  if (m->lx < 1 || m->ly < 1) return fail(SLQ_ERR_ARG, "lx and ly must be >= 1");
  const long n = (long)m->lx * m->ly;
  if (n > 2400) return fail(SLQ_ERR_ARG, "N = lx*ly must be <= 2400");
  if (m->n_slices < 1) return fail(SLQ_ERR_ARG, "n_slices must be >= 1");
  if (m->n_stab < 1) return fail(SLQ_ERR_ARG, "n_stab must be >= 1");
  if (!(m->dtau > 0.0) || !std::isfinite(m->dtau)) return fail(SLQ_ERR_ARG, "dtau must be positive and finite");
  if (!std::isfinite(m->t) || !std::isfinite(m->mu) || !std::isfinite(m->xi))
    return fail(SLQ_ERR_ARG, "t, mu and xi must be finite");
  if (m->chain_prec < SLQ_PREC_FP64 || m->chain_prec > SLQ_PREC_CHECKERBOARD)
    return fail(SLQ_ERR_ARG,
                "chain_prec must be SLQ_PREC_FP64, SLQ_PREC_FP32, SLQ_PREC_BF16, SLQ_PREC_FP64_DENSE or "
                "SLQ_PREC_CHECKERBOARD");
  if (m->chain_prec == SLQ_PREC_CHECKERBOARD && (m->lx % 2 || m->ly % 2))
    return fail(SLQ_ERR_ARG, "the checkerboard split needs even lx and ly");
  return SLQ_OK;
}

int check_model_public(const slq_model* m) { return check_model(m); }

int check_batch(const Plan& p, long batch) {
  if (batch < 0) return fail(SLQ_ERR_ARG, "batch must be >= 0");
  if (batch > p.max_batch) return fail(SLQ_ERR_WORKSPACE, "batch exceeds the plan's max_batch");
  return SLQ_OK;
}

// A launch sequence of one profiled part, bracketed by events when timing is on.
int timed_part(Plan& p, int part, double flops, hipStream_t st, const std::function<int()>& launch) {
  if (!p.prof) return launch();
  std::vector<hipEvent_t>& ev = p.ev[part];
  if (p.ev_used[part] + 2 > ev.size()) {
    for (int k = 0; k < 64; ++k) {
      hipEvent_t e;
      SLQ_HIP(hipEventCreate(&e));
      ev.push_back(e);
    }
  }
  hipEvent_t a = ev[p.ev_used[part]], b = ev[p.ev_used[part] + 1];
  p.ev_used[part] += 2;
  SLQ_HIP(hipEventRecord(a, st));
  int rc = launch();
  SLQ_HIP(hipEventRecord(b, st));
  p.prof_flops[part] += flops;
  return rc;
}

template <typename F>
static int timed_chain(Plan& p, double flops, hipStream_t st, F launch) {
  return timed_part(p, SLQ_PROFILE_CHAIN, flops, st, launch);
}

static int timed_chain_gemm(Plan& p, const GemmArgs& g, hipStream_t st) {
  return timed_chain(p, 2.0 * (double)g.M * g.N * g.K * g.batch, st,
                     [&]() { return launch_gemm(g, false, false, st); });
}

static int timed_chain_kron(Plan& p, const KronArgs& k, hipStream_t st) {
  // circulant lines: 2N (lx + ly) per vector and slice; checkerboard: 7 bond
  // groups of N/2 rotations (6 flops each) and the diagonal factor, 22 N
  const double per = (p.cb ? 22.0 : 2.0 * (double)(p.m.lx + p.m.ly)) * p.n;  // per vector and slice
  const double flops = per * p.n * k.count * k.batch;
  return timed_chain(p, flops, st, [&]() { return launch_kron(p, k, st); });
}

static int timed_chain_lpt(Plan& p, int batch, const void* BT, void* out, int out_f64, const int8_t* s,
                           long strideS, int slice_next, hipStream_t st) {
  return timed_chain(p, 2.0 * (double)p.n * p.n * p.n * batch, st, [&]() {
    return p.m.chain_prec == SLQ_PREC_BF16
               ? launch_bf16t_product(p, batch, BT, out, out_f64, s, strideS, slice_next, st)
               : launch_f32t_product(p, batch, BT, out, out_f64, s, strideS, slice_next, st);
  });
}

static int timed_chain_lp(Plan& p, const LpArgs& g, bool b_is_f64, hipStream_t st) {
  return timed_chain(p, 2.0 * (double)g.M * g.N * g.K * g.batch, st,
                     [&]() { return launch_gemm_lp(g, p.m.chain_prec, b_is_f64, st); });
}

// U D V of the cyclic chain B_{k(L)} ... B_{k(1)} with k(j) = (slice0 + j - 1) mod L + 1,
// i.e. slices slice0+1, ..., L, 1, ..., slice0 multiplied from the right to the left.
int run_chain(Plan& p, int batch, const int8_t* s, int slice0, int32_t* status, hipStream_t st) {
  const int N = p.n, L = p.L, ns = p.m.n_stab;
  const long NN = (long)N * N;
  const long strideS = (long)L * N;
  SLQ_TRY(fill_f64(p.D, (long)batch * N, 1.0, st));
  // V of block k goes to p.V or p.Vt so that the last block's lands in p.V
  const int nblk = (L + ns - 1) / ns;
  double* vnext = (nblk % 2 == 1) ? p.V : p.Vt;
  double* vprev = nullptr;
  GemmArgs g{};
  g.M = N;
  g.N = N;
  g.K = N;
  g.A = p.E;
  g.lda = N;
  g.strideA = 0;
  g.ldb = N;
  g.strideB = NN;
  g.ldc = N;
  g.strideC = NN;
  g.S = s;
  g.strideS = strideS;
  g.inv_scale = 0;
  g.consts = p.consts;
  g.alpha = 1.0;
  g.beta = 0.0;
  g.batch = batch;
  g.cfg = p.gemm_cfg;
  LpArgs h{};
  h.M = N;
  h.N = N;
  h.K = N;
  h.A = p.E32;
  h.lda = N;
  h.ldb = N;
  h.strideB = NN;
  h.ldc = N;
  h.strideC = NN;
  h.S = s;
  h.strideS = strideS;
  h.consts = p.consts;
  h.batch = batch;
  const bool lp = p.m.chain_prec == SLQ_PREC_FP32 || p.m.chain_prec == SLQ_PREC_BF16;
  const bool kron = structured_chain(p);
  for (int j0 = 0; j0 < L; j0 += ns) {
    const int jend = std::min(j0 + ns, L);
    double* cur = p.Xa;
    double* oth = p.Xb;
    if (kron) {
      KronArgs k{};
      k.in = j0 == 0 ? nullptr : p.U;
      k.strideIn = NN;
      k.out = cur;
      k.strideOut = NN;
      k.s = s;
      k.slice0 = (slice0 + j0) % L;
      k.count = jend - j0;
      k.step = 1;
      k.scale = 1;
      k.batch = batch;
      k.norm2 = p.xnorm2;
      k.first_block = p.first_block;
      k.block = j0 / ns;
      SLQ_TRY(timed_chain_kron(p, k, st));
    } else if (!lp) {
      if (j0 == 0) {
        SLQ_TRY(launch_first_slice(p, batch, s, strideS, (slice0 + 0) % L, cur, st));
      } else {
        g.B = p.U;
        g.C = cur;
        g.slice = (slice0 + j0) % L;
        SLQ_TRY(timed_chain_gemm(p, g, st));
      }
      for (int j = j0 + 1; j < jend; ++j) {
        g.B = cur;
        g.C = oth;
        g.slice = (slice0 + j) % L;
        SLQ_TRY(timed_chain_gemm(p, g, st));
        std::swap(cur, oth);
      }
    } else if (lp && N % 8 == 0) {
      // BF16 or FP32 operands, the chain kept as Y^T = (d_next X)^T in the
      // operand type between the slices of the block (two buffers in Xb), X
      // in FP64 after the last one
      const long esz = p.m.chain_prec == SLQ_PREC_BF16 ? 2 : 4;
      char* bt0 = (char*)p.Xb;
      char* bt1 = bt0 + esz * NN * batch;
      SLQ_TRY(launch_bt_prepare(N, batch, j0 == 0 ? nullptr : p.U, NN, s, strideS, (slice0 + j0) % L, p.consts,
                                bt0, p.m.chain_prec, st));
      for (int j = j0; j < jend; ++j) {
        const bool last = j + 1 == jend;
        SLQ_TRY(timed_chain_lpt(p, batch, bt0, last ? (void*)cur : (void*)bt1, last ? 1 : 0, s, strideS,
                                (slice0 + j + 1) % L, st));
        std::swap(bt0, bt1);
      }
    } else {
      // FP32 / BF16 operands, X kept in FP32 (the FP64 buffers hold it), widened before the QR
      float* c32 = (float*)p.Xa;
      float* o32 = (float*)p.Xb;
      if (j0 == 0) {
        SLQ_TRY(launch_first_slice_f32(p, batch, s, strideS, (slice0 + 0) % L, c32, st));
      } else {
        h.B = p.U;
        h.C = c32;
        h.slice = (slice0 + j0) % L;
        SLQ_TRY(timed_chain_lp(p, h, true, st));
      }
      for (int j = j0 + 1; j < jend; ++j) {
        h.B = c32;
        h.C = o32;
        h.slice = (slice0 + j) % L;
        SLQ_TRY(timed_chain_lp(p, h, false, st));
        std::swap(c32, o32);
      }
      cur = (double*)o32;
      SLQ_TRY(launch_widen(c32, cur, NN * batch, st));
    }
    // QR of X diag(D) (R and the explicit Q: (4/3) N^3 + (4/3) N^3 flops per
    // field), then V <- diag(1/D) triu(R) (Pi^T V) (N^3; a permutation only
    // for the first block)
    const double n3 = (double)N * N * N;
    const double stab_flops = batch * (8.0 / 3.0 * n3 + (vprev ? n3 : 0.0));
    SLQ_TRY(timed_part(p, SLQ_PROFILE_STAB, stab_flops, st, [&]() -> int {
      if (N > 64) {
        SLQ_TRY(launch_qr_blocked(p, batch, cur, status, st, kron ? p.xnorm2 : nullptr));
      } else {
        SLQ_TRY(launch_qr(p, batch, cur, status, st));
      }
      if (!vprev) return launch_first_v(p, batch, vnext, st);
      return launch_v_update(p, batch, vprev, vnext, st);
    }));
    vprev = vnext;
    vnext = (vnext == p.V) ? p.Vt : p.V;
  }
  return SLQ_OK;
}

// Byte layout of a plan's workspace, every block 256-byte aligned; with base
// set, the plan's pointers are placed.  Returns the total size.
size_t plan_layout(Plan& p, int32_t flags, char* base) {
  const long N = p.n, NN = N * N, B = p.max_batch;
  const slq_model* model = &p.m;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  const size_t oE32 = take(4 * NN), oE16 = take(2 * NN);
  const size_t oE = take(8 * NN), oEi = take(8 * NN), oTab = take(8 * (2 * (model->lx + model->ly) + 8)),
               oC = take(8 * 8);
  const size_t oXa = take(8 * NN * B), oXb = take(8 * NN * B), oW = take(8 * NN * B), oU = take(8 * NN * B),
               oV = take(8 * NN * B), oVt = take(8 * NN * B);
  const size_t oD = take(8 * N * B), oID = take(8 * N * B), oT = take(8 * (N + 32) * 32 * B),
               oXn = take(8 * N * B);
  const size_t oPerm = take(4 * N * B), oNref = take(4 * B), oSt = take(4 * B), oNref2 = take(4 * B),
               oSt2 = take(4 * B);
  const size_t oSw = take((size_t)p.L * N * B), oDv = take(8 * B), oDv2 = take(8 * B), oIv = take(8 * B);
  const size_t oX = take(8 * N * SWEEP_KD * B), oY = take(8 * N * SWEEP_KD * B), oA = take(8 * SWEEP_KD * B);
  const size_t oFo = take(8 * 64 * B), oFn = take(8 * 64 * B), oSg = take(B), oSg2 = take(B),
               oKw = take(8 * 8 * 64);
  const size_t oFit = take(8 * FIT_ACC_DOUBLES);
  const size_t oQw = take(N > 64 ? 8 * (size_t)qr_workspace_per_field((int)N) * B : 8);
  const size_t oStack = (flags & SLQ_PLAN_SWEEPS) ? take(stack_bytes_for(p, B)) : 0;
  const size_t oNet = (flags & SLQ_PLAN_NET) ? take(net_bytes_for(p)) : 0;
  if (!base) return off;
  char* c = base;
  p.bytes = off;
  p.base = (double*)base;
  p.E = (double*)(c + oE);
  p.Einv = (double*)(c + oEi);
  p.tabs = (double*)(c + oTab);
  p.E32 = (float*)(c + oE32);
  p.E16 = (void*)(c + oE16);
  p.consts = (double*)(c + oC);
  p.Xa = (double*)(c + oXa);
  p.Xb = (double*)(c + oXb);
  p.W = (double*)(c + oW);
  p.U = (double*)(c + oU);
  p.V = (double*)(c + oV);
  p.Vt = (double*)(c + oVt);
  p.D = (double*)(c + oD);
  p.invD = (double*)(c + oID);
  p.Tblk = (double*)(c + oT);
  p.perm = (int32_t*)(c + oPerm);
  p.xnorm2 = (double*)(c + oXn);
  p.nref = (int32_t*)(c + oNref);
  p.status = (int32_t*)(c + oSt);
  p.nref2 = (int32_t*)(c + oNref2);
  p.status2 = (int32_t*)(c + oSt2);
  p.s_work = (int8_t*)(c + oSw);
  p.dvec = (double*)(c + oDv);
  p.dvec2 = (double*)(c + oDv2);
  p.ivec = (int64_t*)(c + oIv);
  p.dX = (double*)(c + oX);
  p.dY = (double*)(c + oY);
  p.dA = (double*)(c + oA);
  p.F_old = (double*)(c + oFo);
  p.F_new = (double*)(c + oFn);
  p.sgn_work = (int8_t*)(c + oSg);
  p.sgn_work2 = (int8_t*)(c + oSg2);
  p.kron_w = (double*)(c + oKw);
  p.fit_acc = (double*)(c + oFit);
  p.qrws = (double*)(c + oQw);
  p.stack = (flags & SLQ_PLAN_SWEEPS) ? (double*)(c + oStack) : nullptr;
  p.stack_batch = (flags & SLQ_PLAN_SWEEPS) ? (int)B : 0;
  p.net_base = (flags & SLQ_PLAN_NET) ? (void*)(c + oNet) : nullptr;
  p.kron_P = kron_line_size(model->lx, model->ly);
  p.cb = model->chain_prec == SLQ_PREC_CHECKERBOARD;
  return off;
}

// Build E, E^{-1}, the structured-product windows and the reduced-precision
// copies of E in the placed workspace, and the host view of the network
// buffers (asynchronous on st).
int plan_init(Plan& p, hipStream_t st) {
  const long NN = (long)p.n * p.n;
  SLQ_TRY(launch_kinetic(p, st));
  SLQ_TRY(launch_kron_windows(p, st));
  if (p.cb) SLQ_TRY(launch_cb_dense(p, st));
  SLQ_TRY(launch_narrow(p.E, p.E32, NN, st));
  SLQ_TRY(launch_to_bf16(p.E32, p.E16, NN, st));
  if (p.net_base) SLQ_TRY(bind_net(p));
  return SLQ_OK;
}

static int weight_or_green(slq_plan* plan, int32_t batch, const int8_t* d_s, double* d_G, double* d_logabs,
                           int8_t* d_sign, int32_t* d_status, hipStream_t st) {
  if (!plan) return fail(SLQ_ERR_ARG, "plan is NULL");
  Plan& p = plan->p;
  SLQ_TRY(check_batch(p, batch));
  if (batch == 0) return SLQ_OK;
  if (!d_s || !d_logabs || !d_sign) return fail(SLQ_ERR_ARG, "d_s, d_logabs and d_sign must not be NULL");
  SLQ_HIP(hipSetDevice(p.device));
  int32_t* status = d_status ? d_status : p.status;
  SLQ_TRY(fill_i32(status, batch, 0, st));
  SLQ_TRY(launch_check_spins(p, batch, d_s, status, st));
  SLQ_TRY(run_chain(p, batch, d_s, 0, status, st));
  return launch_finish(p, batch, d_G, d_logabs, d_sign, status, st);
}

}  // namespace slq

using namespace slq;

extern "C" {

const char* slq_version(void) { return "libslq 0.1 (gfx950)"; }
const char* slq_last_error(void) { return g_err.c_str(); }

int slq_plan_workspace_size(const slq_model* model, int32_t max_batch, int32_t flags, size_t* bytes) {
  if (!bytes) return fail(SLQ_ERR_ARG, "bytes is NULL");
  *bytes = 0;
  SLQ_TRY(check_model(model));
  if (max_batch < 1) return fail(SLQ_ERR_ARG, "max_batch must be >= 1");
  if (flags & ~(SLQ_PLAN_SWEEPS | SLQ_PLAN_NET)) return fail(SLQ_ERR_ARG, "unknown plan flags");
  Plan p{};
  p.m = *model;
  p.n = model->lx * model->ly;
  p.L = model->n_slices;
  p.max_batch = max_batch;
  *bytes = plan_layout(p, flags, nullptr);
  return SLQ_OK;
}

int slq_plan_create(const slq_model* model, int32_t max_batch, int32_t flags, void* d_work, size_t work_bytes,
                    slq_plan** out) {
  if (!out) return fail(SLQ_ERR_ARG, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  SLQ_TRY(slq_plan_workspace_size(model, max_batch, flags, &need));
  if (d_work && work_bytes < need)
    return fail(SLQ_ERR_WORKSPACE, "workspace of " + std::to_string(work_bytes) + " bytes is smaller than the " +
                                       std::to_string(need) + " the plan needs");
  if (d_work && ((uintptr_t)d_work & 255)) return fail(SLQ_ERR_ARG, "d_work must be 256-byte aligned");
  int dev = 0, ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(SLQ_ERR_DEVICE, "no HIP device");
  SLQ_HIP(hipGetDevice(&dev));
  slq_plan* h = new (std::nothrow) slq_plan();
  if (!h) return fail(SLQ_ERR_DEVICE, "host allocation failed");
  Plan& p = h->p;
  p.m = *model;
  p.n = model->lx * model->ly;
  p.L = model->n_slices;
  p.max_batch = max_batch;
  p.device = dev;
  void* base = d_work;
  if (!base) {
    if (hipMalloc(&base, need) != hipSuccess) {
      (void)hipGetLastError();
      delete h;
      return fail(SLQ_ERR_DEVICE, "hipMalloc of " + std::to_string(need) + " bytes failed");
    }
    p.owns_base = true;
  }
  plan_layout(p, flags, (char*)base);
  int rc = plan_init(p, 0);
  if (rc == SLQ_OK && hipDeviceSynchronize() != hipSuccess) rc = fail(SLQ_ERR_DEVICE, "kinetic build failed");
  if (rc != SLQ_OK) {
    release_net(p);
    if (p.owns_base) hipFree(base);
    delete h;
    return rc;
  }
  *out = h;
  return SLQ_OK;
}

int slq_magnetization(slq_plan* plan, int32_t batch, const int8_t* d_s, int64_t* d_M, hipStream_t stream) {
  if (!plan || !d_s || !d_M) return fail(SLQ_ERR_ARG, "NULL argument");
  Plan& p = plan->p;
  SLQ_TRY(check_batch(p, batch));
  if (batch == 0) return SLQ_OK;
  SLQ_HIP(hipSetDevice(p.device));
  k_magnetization<<<batch, 256, 0, stream>>>((long)p.L * p.n, d_s, d_M);
  SLQ_LAUNCHED();
  return SLQ_OK;
}

int slq_profile_enable(slq_plan* plan, int32_t enable) {
  if (!plan) return fail(SLQ_ERR_ARG, "plan is NULL");
  plan->p.prof = enable != 0;
  for (int k = 0; k < 3; ++k) {
    plan->p.ev_used[k] = 0;
    plan->p.prof_flops[k] = 0.0;
  }
  return SLQ_OK;
}

int slq_profile_read_part(slq_plan* plan, int32_t part, double* ms, int64_t* launches, double* flops) {
  if (!plan || !ms || !launches || !flops) return fail(SLQ_ERR_ARG, "NULL argument");
  if (part < SLQ_PROFILE_CHAIN || part > SLQ_PROFILE_FINISH) return fail(SLQ_ERR_ARG, "unknown profile part");
  Plan& p = plan->p;
  SLQ_HIP(hipSetDevice(p.device));
  double tot = 0.0;
  for (size_t k = 0; k + 1 < p.ev_used[part]; k += 2) {
    SLQ_HIP(hipEventSynchronize(p.ev[part][k + 1]));
    float t = 0.f;
    SLQ_HIP(hipEventElapsedTime(&t, p.ev[part][k], p.ev[part][k + 1]));
    tot += t;
  }
  *ms = tot;
  *launches = (int64_t)(p.ev_used[part] / 2);
  *flops = p.prof_flops[part];
  p.ev_used[part] = 0;
  p.prof_flops[part] = 0.0;
  return SLQ_OK;
}

int slq_profile_read(slq_plan* plan, double* ms, int64_t* launches, double* flops) {
  return slq_profile_read_part(plan, SLQ_PROFILE_CHAIN, ms, launches, flops);
}

int slq_plan_destroy(slq_plan* plan) {
  if (!plan) return SLQ_OK;
  hipSetDevice(plan->p.device);
  hipDeviceSynchronize();
  for (int k = 0; k < 3; ++k)
    for (hipEvent_t e : plan->p.ev[k]) hipEventDestroy(e);
  release_net(plan->p);
  if (plan->p.owns_base) hipFree(plan->p.base);
  delete plan;
  return SLQ_OK;
}

int slq_plan_tune(slq_plan* plan, int32_t batch, int32_t* chosen, hipStream_t stream) {
  if (!plan) return fail(SLQ_ERR_ARG, "plan is NULL");
  Plan& p = plan->p;
  SLQ_TRY(check_batch(p, batch));
  if (chosen) *chosen = 0;
  if (batch == 0) return SLQ_OK;
  const bool dense = p.m.chain_prec == SLQ_PREC_FP64_DENSE || (p.m.chain_prec == SLQ_PREC_FP64 && p.kron_P == 0);
  if (dense) {
    SLQ_HIP(hipSetDevice(p.device));
    return tune_chain_gemm(p, batch, stream, nullptr);
  }
  if (p.m.chain_prec != SLQ_PREC_FP64 && !p.cb) return SLQ_OK;
  SLQ_HIP(hipSetDevice(p.device));
  SLQ_TRY(tune_kron(p, batch, stream, nullptr));
  if (chosen) *chosen = p.kron_nb;
  return SLQ_OK;
}

int slq_plan_set_block_width(slq_plan* plan, int32_t width) {
  if (!plan) return fail(SLQ_ERR_ARG, "plan is NULL");
  Plan& p = plan->p;
  if (width == 0) {
    p.kron_nb = 0;
    return SLQ_OK;
  }
  if (!structured_chain(p)) return fail(SLQ_ERR_ARG, "the plan has no structured chain product");
  if (!kron_width_ok(p, width))
    return fail(SLQ_ERR_ARG, "block width must be a power of two <= 32 whose workgroup fits the lattice");
  p.kron_nb = width;
  return SLQ_OK;
}

int slq_plan_bytes(const slq_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return fail(SLQ_ERR_ARG, "NULL argument");
  *bytes = plan->p.bytes;
  return SLQ_OK;
}

int slq_kinetic(slq_plan* plan, int32_t inverse, double* d_out, hipStream_t stream) {
  if (!plan || !d_out) return fail(SLQ_ERR_ARG, "NULL argument");
  Plan& p = plan->p;
  SLQ_HIP(hipSetDevice(p.device));
  return copy_f64(inverse ? p.Einv : p.E, d_out, (long)p.n * p.n, stream);
}

int slq_weight(slq_plan* plan, int32_t batch, const int8_t* d_s, double* d_logabs, int8_t* d_sign,
               int32_t* d_status, hipStream_t stream) {
  return weight_or_green(plan, batch, d_s, nullptr, d_logabs, d_sign, d_status, stream);
}

int slq_green(slq_plan* plan, int32_t batch, const int8_t* d_s, double* d_G, double* d_logabs, int8_t* d_sign,
              int32_t* d_status, hipStream_t stream) {
  if (!d_G) return fail(SLQ_ERR_ARG, "d_G must not be NULL");
  return weight_or_green(plan, batch, d_s, d_G, d_logabs, d_sign, d_status, stream);
}

int slq_udv(slq_plan* plan, int32_t batch, const int8_t* d_s, int32_t slice0, double* d_U, double* d_D,
            double* d_V, int32_t* d_status, hipStream_t stream) {
  if (!plan) return fail(SLQ_ERR_ARG, "plan is NULL");
  Plan& p = plan->p;
  SLQ_TRY(check_batch(p, batch));
  if (batch == 0) return SLQ_OK;
  if (!d_s || !d_U || !d_D || !d_V) return fail(SLQ_ERR_ARG, "NULL device pointer");
  if (slice0 < 0 || slice0 >= p.L) return fail(SLQ_ERR_ARG, "slice0 must be in [0, L)");
  SLQ_HIP(hipSetDevice(p.device));
  int32_t* status = d_status ? d_status : p.status;
  SLQ_TRY(fill_i32(status, batch, 0, stream));
  SLQ_TRY(launch_check_spins(p, batch, d_s, status, stream));
  SLQ_TRY(run_chain(p, batch, d_s, slice0, status, stream));
  const long NN = (long)p.n * p.n;
  SLQ_TRY(copy_f64(p.U, d_U, NN * batch, stream));
  SLQ_TRY(copy_f64(p.D, d_D, (long)p.n * batch, stream));
  SLQ_TRY(copy_f64(p.V, d_V, NN * batch, stream));
  return SLQ_OK;
}

int slq_sweep_local(slq_plan* plan, int32_t batch, int8_t* d_s, double* d_G, double* d_logabs, int8_t* d_sign,
                    int32_t n_sweeps, uint64_t seed, uint64_t sweep0, uint64_t chain0, int64_t* d_accepts,
                    double* d_drift, int32_t* d_status, hipStream_t st) {
  if (!plan) return fail(SLQ_ERR_ARG, "plan is NULL");
  Plan& p = plan->p;
  SLQ_TRY(check_batch(p, batch));
  if (batch == 0 || n_sweeps == 0) return SLQ_OK;
  if (n_sweeps < 0) return fail(SLQ_ERR_ARG, "n_sweeps must be >= 0");
  if (!d_s || !d_G || !d_logabs || !d_sign) return fail(SLQ_ERR_ARG, "NULL device pointer");
  SLQ_HIP(hipSetDevice(p.device));
  int32_t* status = d_status ? d_status : p.status;
  int64_t* acc = d_accepts ? d_accepts : p.ivec;
  double* drift = d_drift ? d_drift : p.dvec2;
  SLQ_TRY(fill_i32(status, batch, 0, st));
  SLQ_TRY(launch_check_spins(p, batch, d_s, status, st));
  SLQ_TRY(fill_i64(acc, batch, 0, st));
  SLQ_TRY(fill_f64(drift, batch, 0.0, st));
  return sweep_stacked(p, batch, d_s, d_G, d_logabs, d_sign, n_sweeps, seed, sweep0, chain0, acc, drift, status, st);
}

}  // extern "C"
