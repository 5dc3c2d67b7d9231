// Groups of independent chains of uneven size (N_c, L_c): one graph-captured
// launch evaluates the exact weight (Eq. 1; and optionally G) of every chain.
//
// Chains with identical models share an internal plan and run as one batch,
// and so do chains on one lattice whose lengths differ by whole stabilisation
// blocks (structured FP64 products): the plan has the longest length and a
// shorter chain starts its stabilised product later.  The fields are gathered
// from the caller's packed layout into the batch,
// evaluated (stabilised chain, QR, LU) and the results scattered back.  The
// whole sequence is recorded once as a HIP graph on the group's own stream
// (per set of caller pointers) and replayed as a single launch; the caller's
// stream is joined with events.  At creation the chain-GEMM tile shape of
// every distinct N is picked by timing the candidate tiles on the device.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "slq_internal.h"

namespace slq {

struct SubPlan {
  slq_plan* plan = nullptr;
  int nb = 0;
  int32_t* d_ids = nullptr;   // [nb] chain index of each batch position
  int64_t* d_soff = nullptr;  // [nb] field offset (bytes) in the caller's packed layout
  int64_t* d_goff = nullptr;  // [nb] G offset (doubles)
  int64_t* d_lead = nullptr;  // [nb] leading slices x N of the batch layout before the chain's own
  int32_t* d_first = nullptr; // [nb] first stabilisation block of each chain
  int lmin = 0;               // shortest chain of the batch (its plan has the longest)
  std::vector<int32_t> ids;   // host copy of d_ids
  int chain0 = 0;             // chains in the batches before this one (random-number stream of the batch)
  // cumulative updates: the batch's current fields and per-chain state
  int8_t* cur = nullptr;      // [nb][L][N]
  double* la = nullptr;       // [nb] log|W|
  double* logA = nullptr;     // [nb]
  int8_t* sg = nullptr;       // [nb] sign
  int8_t* acc = nullptr;      // [nb] accepted
};

struct Group {
  int n = 0;
  int device = 0;
  std::vector<slq_model> models;
  std::vector<int64_t> s_off, g_off;
  std::vector<SubPlan> subs;
  std::vector<int> tuned_n, tuned_kind, tuned_cfg;  // kind 0: chain GEMM tile, 1: structured vectors/workgroup
  std::vector<double> tuned_tflops;
  void* dmem = nullptr;
  void* dstep = nullptr;  // cumulative-update buffers of the batches
  int32_t flags = 0;
  hipStream_t gs = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_fork = nullptr;
  // the sub-batches are dealt to up to kLanes streams (largest estimated work
  // first, each to the least loaded lane); one graph holds every lane as a
  // parallel branch (forked from and joined back to gs during its capture), so
  // an evaluation is one graph launch
  static constexpr int kLanes = 4;
  std::vector<std::vector<int>> lane_subs;
  std::vector<hipStream_t> lane_st;
  std::vector<hipEvent_t> lane_ev;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* key[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};

int check_model_public(const slq_model* m);

// Field of batch position pos: lead[pos] leading +1 entries (slices its chain
// does not have, never multiplied), then the chain's own slices.
__global__ void k_gather(const int8_t* __restrict__ src, const int64_t* __restrict__ soff,
                         const int64_t* __restrict__ lead, long per, int8_t* __restrict__ dst) {
  const int pos = blockIdx.y;
  const long l0 = lead[pos];
  const int8_t* s = src + soff[pos];
  int8_t* d = dst + (long)pos * per;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < per; i += (long)gridDim.x * blockDim.x)
    d[i] = i < l0 ? (int8_t)1 : s[i - l0];
}

__global__ void k_scatter(int nb, const int32_t* __restrict__ ids, const double* __restrict__ la,
                          const int8_t* __restrict__ sg, const int32_t* __restrict__ st, double* __restrict__ out_la,
                          int8_t* __restrict__ out_sg, int32_t* __restrict__ out_st) {
  const int pos = blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= nb) return;
  const int c = ids[pos];
  out_la[c] = la[pos];
  out_sg[c] = sg[pos];
  if (out_st) out_st[c] = st[pos];
}

__global__ void k_gather_state(int nb, const int32_t* __restrict__ ids, const double* __restrict__ la,
                               const int8_t* __restrict__ sg, double* __restrict__ out_la, int8_t* __restrict__ out_sg) {
  const int pos = blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= nb) return;
  out_la[pos] = la[ids[pos]];
  out_sg[pos] = sg[ids[pos]];
}

__global__ void k_scatter_state(int nb, const int32_t* __restrict__ ids, const double* __restrict__ la,
                                const int8_t* __restrict__ sg, const int8_t* __restrict__ acc,
                                const double* __restrict__ logA, const int32_t* __restrict__ st,
                                double* __restrict__ out_la, int8_t* __restrict__ out_sg, int8_t* __restrict__ out_acc,
                                double* __restrict__ out_logA, int32_t* __restrict__ out_st) {
  const int pos = blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= nb) return;
  const int c = ids[pos];
  out_la[c] = la[pos];
  out_sg[c] = sg[pos];
  if (out_acc) out_acc[c] = acc[pos];
  if (out_logA) out_logA[c] = logA[pos];
  if (out_st) out_st[c] = st[pos];
}

__global__ void k_scatter_fields(const int8_t* __restrict__ src, const int64_t* __restrict__ soff, long per,
                                 int8_t* __restrict__ dst) {
  const int pos = blockIdx.y;
  const int8_t* s = src + (long)pos * per;
  int8_t* d = dst + soff[pos];
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < per; i += (long)gridDim.x * blockDim.x) d[i] = s[i];
}

__global__ void k_scatter_g(long NN, const int64_t* __restrict__ goff, const double* __restrict__ G,
                            double* __restrict__ out) {
  const int pos = blockIdx.y;
  const double* s = G + (long)pos * NN;
  double* d = out + goff[pos];
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < NN; i += (long)gridDim.x * blockDim.x) d[i] = s[i];
}

// Chains on one lattice with structured FP64 products whose lengths differ by
// whole stabilisation blocks share a batch: a shorter chain starts its
// stabilised product that many blocks later (U D V = I 1 I until then, which
// the structured product and the QR pass through exactly).
static bool same_but_length(const slq_model& a, const slq_model& b) {
  return a.lx == b.lx && a.ly == b.ly && a.n_stab == b.n_stab && a.t == b.t && a.mu == b.mu && a.dtau == b.dtau &&
         a.xi == b.xi && a.chain_prec == b.chain_prec &&
         ((a.chain_prec == SLQ_PREC_FP64 && kron_line_size(a.lx, a.ly) > 0) ||
          a.chain_prec == SLQ_PREC_CHECKERBOARD) &&
         (a.n_slices - b.n_slices) % a.n_stab == 0;
}

static bool same_model(const slq_model& a, const slq_model& b) {
  return a.lx == b.lx && a.ly == b.ly && a.n_slices == b.n_slices && a.n_stab == b.n_stab && a.t == b.t &&
         a.mu == b.mu && a.dtau == b.dtau && a.xi == b.xi && a.chain_prec == b.chain_prec;
}

// Structured chain products: the fastest number of vectors per workgroup on
// the sub-plan's own buffers and batch size.
static int autotune_kron(Group& g, SubPlan& sp) {
  Plan& p = sp.plan->p;
  float ms = 0.f;
  const int rc = tune_kron(p, sp.nb, g.gs, &ms);
  if (rc != SLQ_OK) return rc;
  g.tuned_n.push_back(p.n);
  g.tuned_kind.push_back(1);
  g.tuned_cfg.push_back(p.kron_nb);
  const int cnt = std::min(p.m.n_stab, p.L);
  const double per = (p.cb ? 22.0 : 2.0 * (double)(p.m.lx + p.m.ly)) * p.n;  // per vector and slice
  g.tuned_tflops.push_back(per * p.n * cnt * sp.nb / (ms * 1e-3) / 1e12);
  return SLQ_OK;
}

// Tune the sub-plan's chain product on its own buffers and batch size: the
// block width of the structured product, or the tile shape of the dense GEMM.
static int autotune(Group& g, SubPlan& sp) {
  Plan& p = sp.plan->p;
  const int N = p.n;
  if (structured_chain(p)) return p.kron_nb > 0 ? SLQ_OK : autotune_kron(g, sp);
  if ((p.m.chain_prec != SLQ_PREC_FP64 && p.m.chain_prec != SLQ_PREC_FP64_DENSE) || p.gemm_cfg >= 0)
    return SLQ_OK;
  float best_ms = 0.f;
  SLQ_TRY(tune_chain_gemm(p, sp.nb, g.gs, &best_ms));
  const int best = p.gemm_cfg;
  g.tuned_n.push_back(N);
  g.tuned_kind.push_back(0);
  g.tuned_cfg.push_back(best);
  g.tuned_tflops.push_back(2.0 * (double)N * N * N * sp.nb * 3 / (best_ms * 1e-3) / 1e12);
  return SLQ_OK;
}

static int enqueue(Group& g, int lane, hipStream_t st, const int8_t* d_s, double* d_G, double* d_logabs,
                   int8_t* d_sign, int32_t* d_status) {
  for (int q : g.lane_subs[lane]) {
    SubPlan& sp = g.subs[q];
    Plan& p = sp.plan->p;
    const long per = (long)p.L * p.n;
    dim3 grid((unsigned)std::max<long>(1, std::min<long>((per + 255) / 256, 256)), sp.nb);
    k_gather<<<grid, 256, 0, st>>>(d_s, sp.d_soff, sp.d_lead, per, p.s_work);
    SLQ_LAUNCHED();
    int rc = fill_i32(p.status, sp.nb, 0, st);
    if (rc == SLQ_OK) rc = launch_check_spins(p, sp.nb, p.s_work, p.status, st);
    if (rc == SLQ_OK) rc = run_chain(p, sp.nb, p.s_work, 0, p.status, st);
    if (rc == SLQ_OK) rc = launch_finish(p, sp.nb, d_G ? p.Xa : nullptr, p.dvec, p.sgn_work, p.status, st);
    if (rc != SLQ_OK) return rc;
    k_scatter<<<(sp.nb + 63) / 64, 64, 0, st>>>(sp.nb, sp.d_ids, p.dvec, p.sgn_work, p.status, d_logabs, d_sign,
                                                 d_status);
    SLQ_LAUNCHED();
    if (d_G) {
      const long NN = (long)p.n * p.n;
      dim3 gg((unsigned)std::max<long>(1, std::min<long>((NN + 255) / 256, 256)), sp.nb);
      k_scatter_g<<<gg, 256, 0, st>>>(NN, sp.d_goff, p.Xa, d_G);
      SLQ_LAUNCHED();
    }
  }
  return SLQ_OK;
}

static void drop_graph(Group& g) {
  if (g.exec) hipGraphExecDestroy(g.exec);
  if (g.graph) hipGraphDestroy(g.graph);
  g.exec = nullptr;
  g.graph = nullptr;
}

// Record the evaluation as one graph: the capture starts on gs, forks to the
// lane streams through ev_fork and joins them back through their events.
static int record_graph(Group& g, const int8_t* d_s, double* d_G, double* d_logabs, int8_t* d_sign,
                        int32_t* d_status) {
  SLQ_HIP(hipStreamBeginCapture(g.gs, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipEventRecord(g.ev_fork, g.gs);
  int rc = e == hipSuccess ? SLQ_OK : SLQ_ERR_DEVICE;
  for (size_t k = 0; k < g.lane_st.size(); ++k) {
    hipStream_t ls = g.lane_st[k];
    if (e == hipSuccess) e = hipStreamWaitEvent(ls, g.ev_fork, 0);
    if (e == hipSuccess && rc == SLQ_OK) rc = enqueue(g, (int)k, ls, d_s, d_G, d_logabs, d_sign, d_status);
    if (e == hipSuccess) e = hipEventRecord(g.lane_ev[k], ls);
    if (e == hipSuccess) e = hipStreamWaitEvent(g.gs, g.lane_ev[k], 0);
  }
  hipGraph_t graph = nullptr;
  const hipError_t ee = hipStreamEndCapture(g.gs, &graph);
  if (rc != SLQ_OK || e != hipSuccess || ee != hipSuccess) {
    if (graph) hipGraphDestroy(graph);
    if (rc != SLQ_OK) return rc;
    set_error(std::string("graph capture of the group: ") + hipGetErrorString(e != hipSuccess ? e : ee));
    return SLQ_ERR_DEVICE;
  }
  g.graph = graph;
  SLQ_HIP(hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0));
  return SLQ_OK;
}

static int group_eval(Group& g, const int8_t* d_s, double* d_G, double* d_logabs, int8_t* d_sign, int32_t* d_status,
                      hipStream_t stream) {
  SLQ_HIP(hipSetDevice(g.device));
  SLQ_HIP(hipEventRecord(g.ev_in, stream));
  const void* key[5] = {d_s, d_G, d_logabs, d_sign, d_status};
  if (!g.exec || memcmp(key, g.key, sizeof(key)) != 0) {
    drop_graph(g);
    memset(g.key, 0, sizeof(g.key));
    // one eager pass on the lanes (sets the kernel attributes), then the capture
    for (size_t k = 0; k < g.lane_st.size(); ++k) {
      hipStream_t ls = g.lane_st[k];
      SLQ_HIP(hipStreamWaitEvent(ls, g.ev_in, 0));
      SLQ_TRY(enqueue(g, (int)k, ls, d_s, d_G, d_logabs, d_sign, d_status));
      SLQ_HIP(hipEventRecord(g.lane_ev[k], ls));
      SLQ_HIP(hipStreamWaitEvent(g.gs, g.lane_ev[k], 0));
    }
    SLQ_TRY(record_graph(g, d_s, d_G, d_logabs, d_sign, d_status));
    memcpy(g.key, key, sizeof(key));
  }
  SLQ_HIP(hipStreamWaitEvent(g.gs, g.ev_in, 0));
  SLQ_HIP(hipGraphLaunch(g.exec, g.gs));
  SLQ_HIP(hipEventRecord(g.ev_out, g.gs));
  SLQ_HIP(hipStreamWaitEvent(stream, g.ev_out, 0));
  return SLQ_OK;
}

static void release(Group& g) {
  hipSetDevice(g.device);
  if (g.gs) hipStreamSynchronize(g.gs);
  for (hipStream_t ls : g.lane_st)
    if (ls) hipStreamSynchronize(ls);
  drop_graph(g);
  for (hipEvent_t e : g.lane_ev)
    if (e) hipEventDestroy(e);
  for (hipStream_t ls : g.lane_st)
    if (ls) hipStreamDestroy(ls);
  for (SubPlan& sp : g.subs) slq_plan_destroy(sp.plan);
  if (g.dmem) hipFree(g.dmem);
  if (g.dstep) hipFree(g.dstep);
  if (g.ev_in) hipEventDestroy(g.ev_in);
  if (g.ev_out) hipEventDestroy(g.ev_out);
  if (g.ev_fork) hipEventDestroy(g.ev_fork);
  if (g.gs) hipStreamDestroy(g.gs);
  g = Group();
}

}  // namespace slq

struct slq_group {
  slq::Group g;
};

using namespace slq;

extern "C" {

int slq_group_create(const slq_model* models, int32_t n_chains, slq_group** out) {
  return slq_group_create_flags(models, n_chains, 0, out);
}

int slq_group_create_flags(const slq_model* models, int32_t n_chains, int32_t flags, slq_group** out) {
  if (flags & ~SLQ_GROUP_EXACT_BATCHES) {
    set_error("unknown group flags");
    return SLQ_ERR_ARG;
  }
  if (!models || !out || n_chains < 1) {
    set_error("models, out and n_chains >= 1 are required");
    return SLQ_ERR_ARG;
  }
  *out = nullptr;
  for (int c = 0; c < n_chains; ++c) {
    int rc = check_model_public(&models[c]);
    if (rc != SLQ_OK) return rc;
  }
  slq_group* h = new (std::nothrow) slq_group();
  if (!h) {
    set_error("host allocation failed");
    return SLQ_ERR_DEVICE;
  }
  Group& g = h->g;
  g.flags = flags;
  g.n = n_chains;
  g.models.assign(models, models + n_chains);
  if (hipGetDevice(&g.device) != hipSuccess) {
    delete h;
    set_error("no HIP device");
    return SLQ_ERR_DEVICE;
  }
  g.s_off.resize(n_chains + 1);
  g.g_off.resize(n_chains + 1);
  g.s_off[0] = 0;
  g.g_off[0] = 0;
  for (int c = 0; c < n_chains; ++c) {
    const long N = (long)models[c].lx * models[c].ly;
    g.s_off[c + 1] = g.s_off[c] + (long)models[c].n_slices * N;
    g.g_off[c + 1] = g.g_off[c] + N * N;
  }
  // sub-plans in order of first appearance: identical models, or models that
  // differ only in their length by whole stabilisation blocks (the batch's
  // plan has the longest); rep[k] is the longest member
  std::vector<std::vector<int>> members;
  std::vector<int> rep;
  for (int c = 0; c < n_chains; ++c) {
    int k = -1;
    for (size_t q = 0; q < rep.size() && k < 0; ++q)
      if (same_model(models[rep[q]], models[c]) ||
          (!(flags & SLQ_GROUP_EXACT_BATCHES) && same_but_length(models[rep[q]], models[c])))
        k = (int)q;
    if (k < 0) {
      rep.push_back(c);
      members.emplace_back();
      k = (int)rep.size() - 1;
    }
    members[k].push_back(c);
    if (models[c].n_slices > models[rep[k]].n_slices) rep[k] = c;
  }
  size_t bytes = 0;
  for (auto& mset : members) bytes += mset.size() * (4 + 8 + 8 + 8 + 4) + 2 * 64;
  if (hipMalloc(&g.dmem, bytes) != hipSuccess) {
    delete h;
    set_error("hipMalloc failed");
    return SLQ_ERR_DEVICE;
  }
  char* dp = (char*)g.dmem;
  int rc = SLQ_OK;
  for (size_t q = 0; q < members.size() && rc == SLQ_OK; ++q) {
    SubPlan sp;
    sp.nb = (int)members[q].size();
    rc = slq_plan_create(&models[rep[q]], sp.nb, 0, nullptr, 0, &sp.plan);
    if (rc != SLQ_OK) break;
    std::vector<int32_t> ids(members[q].begin(), members[q].end()), first(sp.nb);
    std::vector<int64_t> so(sp.nb), go(sp.nb), lead(sp.nb);
    const slq_model& mr = models[rep[q]];
    const long N = (long)mr.lx * mr.ly;
    bool varied = false;
    sp.lmin = mr.n_slices;
    for (int i = 0; i < sp.nb; ++i) {
      const int dl = mr.n_slices - models[ids[i]].n_slices;  // a multiple of n_stab
      so[i] = g.s_off[ids[i]];
      go[i] = g.g_off[ids[i]];
      lead[i] = (int64_t)dl * N;
      first[i] = dl / mr.n_stab;
      varied = varied || dl != 0;
      sp.lmin = std::min(sp.lmin, models[ids[i]].n_slices);
    }
    sp.d_soff = (int64_t*)dp;
    dp += 8 * sp.nb;
    sp.d_goff = (int64_t*)dp;
    dp += 8 * sp.nb;
    sp.d_lead = (int64_t*)dp;
    dp += 8 * sp.nb;
    sp.d_ids = (int32_t*)dp;
    dp += 4 * sp.nb + (64 - (4 * sp.nb) % 64) % 64;
    sp.d_first = (int32_t*)dp;
    dp += 4 * sp.nb + (64 - (4 * sp.nb) % 64) % 64;
    if (hipMemcpy(sp.d_soff, so.data(), 8 * sp.nb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(sp.d_goff, go.data(), 8 * sp.nb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(sp.d_lead, lead.data(), 8 * sp.nb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(sp.d_ids, ids.data(), 4 * sp.nb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(sp.d_first, first.data(), 4 * sp.nb, hipMemcpyHostToDevice) != hipSuccess) {
      set_error("hipMemcpy failed");
      rc = SLQ_ERR_DEVICE;
    }
    if (varied) sp.plan->p.first_block = sp.d_first;
    sp.ids = ids;
    sp.chain0 = g.subs.empty() ? 0 : g.subs.back().chain0 + g.subs.back().nb;
    g.subs.push_back(sp);
  }
  // buffers of the cumulative updates: each batch's current fields and state
  if (rc == SLQ_OK) {
    size_t sb = 0;
    auto align = [](size_t x) { return (x + 255) / 256 * 256; };
    for (SubPlan& sp : g.subs) {
      const Plan& p = sp.plan->p;
      sb += align((size_t)sp.nb * p.L * p.n) + 2 * align(8 * (size_t)sp.nb) + 2 * align((size_t)sp.nb);
    }
    if (hipMalloc(&g.dstep, sb) != hipSuccess) {
      set_error("hipMalloc failed");
      rc = SLQ_ERR_DEVICE;
    } else {
      char* q = (char*)g.dstep;
      for (SubPlan& sp : g.subs) {
        const Plan& p = sp.plan->p;
        sp.cur = (int8_t*)q;
        q += align((size_t)sp.nb * p.L * p.n);
        sp.la = (double*)q;
        q += align(8 * (size_t)sp.nb);
        sp.logA = (double*)q;
        q += align(8 * (size_t)sp.nb);
        sp.sg = (int8_t*)q;
        q += align((size_t)sp.nb);
        sp.acc = (int8_t*)q;
        q += align((size_t)sp.nb);
      }
    }
  }
  if (rc == SLQ_OK && (hipStreamCreateWithFlags(&g.gs, hipStreamNonBlocking) != hipSuccess ||
                       hipEventCreateWithFlags(&g.ev_in, hipEventDisableTiming) != hipSuccess ||
                       hipEventCreateWithFlags(&g.ev_out, hipEventDisableTiming) != hipSuccess ||
                       hipEventCreateWithFlags(&g.ev_fork, hipEventDisableTiming) != hipSuccess)) {
    set_error("stream/event creation failed");
    rc = SLQ_ERR_DEVICE;
  }
  if (rc == SLQ_OK) {  // lanes: estimated work per sub-batch ~ fields x (stabilisations N^3 + products N^2 (lx+ly) L)
    const int nl = std::min<int>(Group::kLanes, (int)g.subs.size());
    std::vector<double> work(g.subs.size()), load(nl, 0.0);
    std::vector<int> order(g.subs.size());
    for (size_t q = 0; q < g.subs.size(); ++q) {
      const slq_model& m = g.subs[q].plan->p.m;
      const double N = (double)m.lx * m.ly;
      const double nst = (double)((m.n_slices + m.n_stab - 1) / m.n_stab);
      work[q] = g.subs[q].nb * (nst * N * N * N + N * N * (m.lx + m.ly) * m.n_slices);
      order[q] = (int)q;
    }
    std::sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
    g.lane_subs.assign(nl, {});
    for (int q : order) {
      const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      g.lane_subs[k].push_back(q);
      load[k] += work[q];
    }
    g.lane_st.assign(nl, nullptr);
    g.lane_ev.assign(nl, nullptr);
    for (int k = 0; k < nl && rc == SLQ_OK; ++k)
      if (hipStreamCreateWithFlags(&g.lane_st[k], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&g.lane_ev[k], hipEventDisableTiming) != hipSuccess) {
        set_error("stream/event creation failed");
        rc = SLQ_ERR_DEVICE;
      }
  }
  // autotune the chain product once per lattice, on the largest batch of that
  // lattice, and share the choice with its other sub-plans
  auto same_lattice = [&](size_t r, size_t q) {
    const slq_model &a = g.subs[r].plan->p.m, &c = g.subs[q].plan->p.m;
    return a.lx == c.lx && a.ly == c.ly && a.chain_prec == c.chain_prec;
  };
  for (size_t q = 0; q < g.subs.size() && rc == SLQ_OK; ++q) {
    size_t pick = q;
    for (size_t r = 0; r < g.subs.size(); ++r)
      if (same_lattice(r, q) && g.subs[r].nb > g.subs[pick].nb) pick = r;
    rc = autotune(g, g.subs[pick]);
    Plan& tp = g.subs[pick].plan->p;
    g.subs[q].plan->p.kron_nb = tp.kron_nb;
    g.subs[q].plan->p.gemm_cfg = tp.gemm_cfg;
  }
  if (rc == SLQ_OK && hipStreamSynchronize(g.gs) != hipSuccess) {
    set_error("autotuning failed");
    rc = SLQ_ERR_DEVICE;
  }
  if (rc != SLQ_OK) {
    release(h->g);
    delete h;
    return rc;
  }
  *out = h;
  return SLQ_OK;
}

int slq_group_destroy(slq_group* grp) {
  if (!grp) return SLQ_OK;
  release(grp->g);
  delete grp;
  return SLQ_OK;
}

int slq_group_layout(const slq_group* grp, int64_t* s_off, int64_t* g_off) {
  if (!grp || !s_off) {
    set_error("NULL argument");
    return SLQ_ERR_ARG;
  }
  const Group& g = grp->g;
  for (int c = 0; c <= g.n; ++c) {
    s_off[c] = g.s_off[c];
    if (g_off) g_off[c] = g.g_off[c];
  }
  return SLQ_OK;
}

int slq_group_describe(const slq_group* grp, char* buf, size_t len) {
  if (!grp || !buf || len == 0) {
    set_error("NULL argument");
    return SLQ_ERR_ARG;
  }
  const Group& g = grp->g;
  std::string s = "{\"chains\": " + std::to_string(g.n) + ", \"batches\": [";
  for (size_t q = 0; q < g.subs.size(); ++q) {
    const Plan& p = g.subs[q].plan->p;
    s += (q ? ", " : "") + std::string("{\"N\": ") + std::to_string(p.n) + ", \"L\": " + std::to_string(p.L) +
         ", \"L_min\": " + std::to_string(g.subs[q].lmin) + ", \"chains\": " + std::to_string(g.subs[q].nb) + "}";
  }
  s += "], \"lanes\": [";
  for (size_t k = 0; k < g.lane_subs.size(); ++k) {
    s += k ? ", [" : "[";
    for (size_t i = 0; i < g.lane_subs[k].size(); ++i) s += (i ? ", " : "") + std::to_string(g.lane_subs[k][i]);
    s += "]";
  }
  s += "], \"tuned\": [";
  for (size_t q = 0; q < g.tuned_n.size(); ++q) {
    char tmp[128];
    snprintf(tmp, sizeof(tmp), "%s{\"N\": %d, \"kind\": \"%s\", \"cfg\": %d, \"tflops\": %.3f}", q ? ", " : "",
             g.tuned_n[q], g.tuned_kind[q] ? "kron_nb" : "gemm_cfg", g.tuned_cfg[q], g.tuned_tflops[q]);
    s += tmp;
  }
  s += "]}";
  if (s.size() + 1 > len) {
    set_error("buffer too small");
    return SLQ_ERR_ARG;
  }
  memcpy(buf, s.c_str(), s.size() + 1);
  return SLQ_OK;
}

int slq_group_batches(const slq_group* grp, int32_t* n_batches) {
  if (!grp || !n_batches) {
    set_error("NULL argument");
    return SLQ_ERR_ARG;
  }
  *n_batches = (int32_t)grp->g.subs.size();
  return SLQ_OK;
}

int slq_group_batch(slq_group* grp, int32_t k, slq_plan** plan, int32_t* n_chains, int32_t* chain_ids) {
  if (!grp || !plan || !n_chains) {
    set_error("NULL argument");
    return SLQ_ERR_ARG;
  }
  const Group& g = grp->g;
  if (k < 0 || k >= (int32_t)g.subs.size()) {
    set_error("batch index out of range");
    return SLQ_ERR_ARG;
  }
  const SubPlan& sp = g.subs[k];
  *plan = sp.plan;
  *n_chains = sp.nb;
  if (chain_ids) memcpy(chain_ids, sp.ids.data(), sizeof(int32_t) * sp.nb);
  return SLQ_OK;
}

int slq_group_cumulative_step(slq_group* grp, slq_eff* const* effs, int32_t eff_sweeps, uint64_t seed, uint64_t step,
                              int8_t* d_s, double* d_logabs, int8_t* d_sign, int8_t* d_accepted, double* d_logA,
                              int32_t* d_status, hipStream_t stream) {
  if (!grp || !effs || !d_s || !d_logabs || !d_sign) {
    set_error("NULL argument");
    return SLQ_ERR_ARG;
  }
  Group& g = grp->g;
  if (eff_sweeps < 0) {
    set_error("eff_sweeps must be >= 0");
    return SLQ_ERR_ARG;
  }
  for (size_t q = 0; q < g.subs.size(); ++q) {
    if (g.subs[q].lmin != g.subs[q].plan->p.L) {
      set_error("the group batches chains of different lengths; create it with SLQ_GROUP_EXACT_BATCHES");
      return SLQ_ERR_ARG;
    }
    if (!effs[q]) {
      set_error("one effective model per batch is required");
      return SLQ_ERR_ARG;
    }
  }
  SLQ_HIP(hipSetDevice(g.device));
  SLQ_HIP(hipEventRecord(g.ev_in, stream));
  for (size_t k = 0; k < g.lane_st.size(); ++k) {
    hipStream_t ls = g.lane_st[k];
    SLQ_HIP(hipStreamWaitEvent(ls, g.ev_in, 0));
    for (int q : g.lane_subs[k]) {
      SubPlan& sp = g.subs[q];
      Plan& p = sp.plan->p;
      const long per = (long)p.L * p.n;
      const dim3 fgrid((unsigned)std::max<long>(1, std::min<long>((per + 255) / 256, 256)), sp.nb);
      const unsigned sgrid = (unsigned)((sp.nb + 63) / 64);
      int32_t classes = 0;
      SLQ_TRY(slq_eff_classes(effs[q], &classes));
      k_gather<<<fgrid, 256, 0, ls>>>(d_s, sp.d_soff, sp.d_lead, per, sp.cur);
      SLQ_LAUNCHED();
      k_gather_state<<<sgrid, 64, 0, ls>>>(sp.nb, sp.d_ids, d_logabs, d_sign, sp.la, sp.sg);
      SLQ_LAUNCHED();
      SLQ_TRY(slq_cumulative_step(sp.plan, effs[q], sp.nb, sp.cur, sp.la, sp.sg, eff_sweeps * classes, seed, step,
                                  (uint64_t)sp.chain0, sp.acc, sp.logA, p.status, ls));
      k_scatter_fields<<<fgrid, 256, 0, ls>>>(sp.cur, sp.d_soff, per, d_s);
      SLQ_LAUNCHED();
      k_scatter_state<<<sgrid, 64, 0, ls>>>(sp.nb, sp.d_ids, sp.la, sp.sg, sp.acc, sp.logA, p.status, d_logabs,
                                            d_sign, d_accepted, d_logA, d_status);
      SLQ_LAUNCHED();
    }
    SLQ_HIP(hipEventRecord(g.lane_ev[k], ls));
    SLQ_HIP(hipStreamWaitEvent(stream, g.lane_ev[k], 0));
  }
  return SLQ_OK;
}

int slq_group_weight(slq_group* grp, const int8_t* d_s, double* d_logabs, int8_t* d_sign, int32_t* d_status,
                     hipStream_t stream) {
  if (!grp || !d_s || !d_logabs || !d_sign) {
    set_error("NULL argument");
    return SLQ_ERR_ARG;
  }
  return group_eval(grp->g, d_s, nullptr, d_logabs, d_sign, d_status, stream);
}

int slq_group_green(slq_group* grp, const int8_t* d_s, double* d_G, double* d_logabs, int8_t* d_sign,
                    int32_t* d_status, hipStream_t stream) {
  if (!grp || !d_s || !d_G || !d_logabs || !d_sign) {
    set_error("NULL argument");
    return SLQ_ERR_ARG;
  }
  return group_eval(grp->g, d_s, d_G, d_logabs, d_sign, d_status, stream);
}

}  // extern "C"
