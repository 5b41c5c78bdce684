// api.cpp - the C ABI (include/tnapprox.h): handles, plan cache, device buffers, launches.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.hpp"
#include "planner.hpp"
#include "tnapprox.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) return fail(TN_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// A run of ops executed one way: kind 0 = ops [first, last) by one workgroup,
// 1 = GEMM op `first` over `blocks` workgroups, 2 = RESCALE op `first` likewise.
struct Seg {
  int kind;
  int64_t first, last;
  int blocks;
  bool piped;        // kind 1: offsets fit the pipelined chip-wide kernel
  int64_t split_bytes = 0;   // kind 1: scratch of the split forms' operand planes
  int split_blocks = 0;      // kind 1: workgroups of the split forms' operand pass
  int kchunks = 1;           // kind 1, FP64 tiled: parts of K (split K), scratch kpart doubles
  int64_t kpart = 0;
  int stream_k = 0;          // kind 1, FP64: streamed (K class), over stream_blocks workgroups
  int stream_blocks = 0;
};

struct DevPlan {
  tn::Plan plan;
  std::vector<Seg> segs;     // empty: the whole network fits one workgroup's pass
  tn::Op *d_ops = nullptr;
  int32_t *d_tab = nullptr;
  // the launches of `segs`, captured as a HIP graph once per set of launch parameters
  // (keyed by them; the network's descriptor is read at run time). Graphs are kept, not
  // re-captured, when a call switches between parameter sets.
  std::map<std::vector<char>, hipGraphExec_t> gexecs;
  ~DevPlan() {
    for (auto &kv : gexecs) (void)hipGraphExecDestroy(kv.second);
    if (d_ops) (void)hipFree(d_ops);
    if (d_tab) (void)hipFree(d_tab);
  }
};

using PlanKey = std::tuple<std::vector<std::vector<int32_t>>, int32_t, int32_t>;

int check_device() {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return fail(TN_EDEVICE, "no HIP device visible");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(TN_EDEVICE, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
  return TN_OK;
}

int read_path(const tn_path *path, int32_t nt, std::vector<std::vector<int32_t>> &slices) {
  if (!path || path->n_slices < 1 || !path->slice_ptr || !path->slice_vertices)
    return fail(TN_EINVAL, "path is empty or has null arrays");
  slices.assign(path->n_slices, {});
  if (path->slice_ptr[0] != 0) return fail(TN_EINVAL, "slice_ptr[0] must be 0");
  for (int32_t s = 0; s < path->n_slices; ++s) {
    int32_t b = path->slice_ptr[s], e = path->slice_ptr[s + 1];
    if (e < b || e > nt) return fail(TN_EINVAL, "slice_ptr is not non-decreasing within the tensor count");
    slices[s].assign(path->slice_vertices + b, path->slice_vertices + e);
  }
  if (path->slice_ptr[path->n_slices] != nt) return fail(TN_EINVAL, "slices do not list every tensor exactly once");
  return TN_OK;
}

}  // namespace

struct tn_net_s {
  tn::Graph g;
  tn::NetScalars last{};     // device scalars of the last contraction
  double *d_const = nullptr;
  double *d_ws = nullptr;
  int64_t ws_cap = 0;
  tn::NetScalars *d_sc = nullptr;
  std::map<PlanKey, std::unique_ptr<DevPlan>> plans;
  // for networks run op by op: a device copy of the network's descriptor, the grid
  // scratch and a stream to capture the op launches on (all kept while the handle lives)
  tn::NetDev *d_nd = nullptr;
  double *d_part = nullptr;
  unsigned short *d_split = nullptr;   // split forms: operand planes of the chip-wide GEMMs
  int64_t split_cap = 0;
  double *d_kpart = nullptr;           // split-K partial products of the chip-wide GEMMs
  int64_t kpart_cap = 0;
  hipStream_t cap_stream = nullptr;
  ~tn_net_s() {
    plans.clear();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (d_nd) (void)hipFree(d_nd);
    if (d_part) (void)hipFree(d_part);
    if (d_split) (void)hipFree(d_split);
    if (d_kpart) (void)hipFree(d_kpart);
    if (d_const) (void)hipFree(d_const);
    if (d_ws) (void)hipFree(d_ws);
    if (d_sc) (void)hipFree(d_sc);
  }
};

struct tn_model_s {
  float *d_w = nullptr, *d_m = nullptr, *d_v = nullptr, *d_loss = nullptr;
  long long t = 0;                 // Adam steps taken
  ~tn_model_s() {
    (void)hipFree(d_w); (void)hipFree(d_m); (void)hipFree(d_v); (void)hipFree(d_loss);
  }
};

struct tn_dataset_s {
  float *d_x = nullptr, *d_y = nullptr;
  int *d_count = nullptr;
  int64_t cap = 0;
  ~tn_dataset_s() {
    (void)hipFree(d_x); (void)hipFree(d_y); (void)hipFree(d_count);
  }
};

namespace {

int64_t box_static(const tn::Box &b) {
  int64_t n = b.rest;
  for (int d = 0; d < b.nd; ++d) n *= b.cap[d];
  return n;
}

// A network with an op whose output exceeds 2^21 elements (or a GEMM above 2^32 flops)
// runs op by op. In such a network every op with an output of at least 2^13 elements
// (or a GEMM of at least 2^24 flops) runs over the whole chip, the rest in single-
// workgroup stretches between them. Networks without such ops keep the one-pass
// interpreter.
void make_segments(DevPlan &dp) {
  constexpr int64_t kBigOut = int64_t(1) << 21, kBigFlops = int64_t(1) << 32;
  constexpr int64_t kGridOut = int64_t(1) << 13, kGridFlops = int64_t(1) << 24;
  const auto &ops = dp.plan.ops;
  auto out_of = [](const tn::Op &op) -> int64_t {
    if (op.kind == tn::OP_GEMM) return int64_t(op.am.n) * op.bn.n;
    if (op.kind == tn::OP_RESCALE) return box_static(op.bm) * box_static(op.bnb);
    return 0;
  };
  bool any = false;
  for (const tn::Op &op : ops) {
    const int64_t out = out_of(op);
    if (out >= kBigOut || (op.kind == tn::OP_GEMM && 2 * out * op.K >= kBigFlops)) any = true;
  }
  if (!any) return;
  std::vector<Seg> segs;
  for (int64_t i = 0; i < int64_t(ops.size()); ++i) {
    const tn::Op &op = ops[size_t(i)];
    const int64_t out = out_of(op);
    int kind = 0, blocks = 0;
    bool piped = false;
    if (op.kind == tn::OP_GEMM && (out >= kGridOut || 2 * out * op.K >= kGridFlops)) {
      kind = 1;
      blocks = int(std::min<int64_t>(tn::kGridBlocks, ((op.am.n + 63) / 64) * ((op.bn.n + 63) / 64)));
      piped = int64_t(op.am.n) + op.K <= int64_t(tn::kGridOffsetDoubles) && out < (int64_t(1) << 31);
    } else if (op.kind == tn::OP_RESCALE && out >= kGridOut) {
      kind = 2;
      blocks = int(std::min<int64_t>(tn::kGridBlocks, (out + 2047) / 2048));
    }
    if (kind) {
      segs.push_back(Seg{kind, i, i + 1, std::max(blocks, 1), piped});
      if (kind == 1) {
        Seg &sg = segs.back();
        sg.split_bytes = tn::split_scratch_bytes(op.am.n, op.bn.n, op.K);
        sg.split_blocks = tn::split_grid_blocks(op.am.n, op.bn.n, op.K);
        if (!piped) {
          sg.kchunks = tn::grid_kchunks(op.am.n, op.bn.n, op.K);
          sg.kpart = tn::grid_kpart_doubles(op.am.n, op.bn.n, op.K);
        }
        sg.stream_k = tn::stream_kclass(op.am.n, op.bn.n, op.K);
        sg.stream_blocks = tn::stream_blocks(op.bn.n);
      }
    } else if (!segs.empty() && segs.back().kind == 0) {
      segs.back().last = i + 1;
    } else {
      segs.push_back(Seg{0, i, i + 1, 1, false});
    }
  }
  dp.segs = std::move(segs);
}

// The plan of (slices, chi, env) on the handle, built on first use. `device`: also give
// it device copies of its op list and index tables (the allocation-free entry point
// passes false and copies them into its scratch instead).
int get_plan(tn_net net, const std::vector<std::vector<int32_t>> &slices, int32_t chi, int32_t env,
             DevPlan **out, bool device = true) {
  PlanKey key{slices, chi, env};
  auto it = net->plans.find(key);
  DevPlan *dp = nullptr;
  if (it != net->plans.end()) {
    dp = it->second.get();
  } else {
    auto np = std::make_unique<DevPlan>();
    tn::PlanArgs pa;
    pa.slices = slices;
    pa.chi = chi;
    pa.env = env;
    bool unsup = false;
    std::string err = tn::make_plan(net->g, pa, np->plan, &unsup);
    if (!err.empty()) return fail(unsup ? TN_EUNSUPPORTED : TN_EINVAL, err);
    make_segments(*np);
    dp = np.get();
    net->plans.emplace(std::move(key), std::move(np));
  }
  if (device && !dp->d_ops) {
    size_t ob = dp->plan.ops.size() * sizeof(tn::Op), tb = std::max<size_t>(1, dp->plan.tables.size()) * 4;
    if (!dp->d_tab && hipMalloc(&dp->d_tab, tb) != hipSuccess) return fail(TN_ENOMEM, "device allocation for the plan failed");
    if (!dp->plan.tables.empty())
      HIP_TRY(hipMemcpy(dp->d_tab, dp->plan.tables.data(), dp->plan.tables.size() * 4, hipMemcpyHostToDevice));
    tn::Op *ops = nullptr;                 // set last: a plan with d_ops has both copies
    if (hipMalloc(&ops, std::max<size_t>(ob, 64)) != hipSuccess) return fail(TN_ENOMEM, "device allocation for the plan failed");
    dp->d_ops = ops;
    if (ob) HIP_TRY(hipMemcpy(dp->d_ops, dp->plan.ops.data(), ob, hipMemcpyHostToDevice));
  }
  *out = dp;
  return TN_OK;
}

int ensure_ws(tn_net net, int64_t doubles) {
  doubles = std::max<int64_t>(doubles, 32);
  if (net->ws_cap >= doubles) return TN_OK;
  if (net->d_ws) (void)hipFree(net->d_ws);
  net->d_ws = nullptr;
  net->ws_cap = 0;
  if (hipMalloc(&net->d_ws, size_t(doubles) * 8) != hipSuccess)
    return fail(TN_ENOMEM, "workspace allocation of " + std::to_string(doubles * 8) + " bytes failed");
  net->ws_cap = doubles;
  return TN_OK;
}

// Default rank rule: keep eigenvalues above 1e-12 of the largest (what an FP64 solve
// resolves), never cut at a relative gap of 10% or less.
constexpr double kTauRel = 1e-12, kTauDeg = 0.1;

tn_options defaults() {
  tn_options o;
  std::memset(&o, 0, sizeof(o));
  o.precision = TN_FP64;
  o.eig = TN_EIG_EXACT;
  o.residual_tol = 1e-6;
  o.tau_rel = kTauRel;
  o.tau_deg = kTauDeg;
  o.hip_stream = nullptr;
  return o;
}

// The launch parameters as a byte key, field by field (no padding bytes).
void key_put(std::vector<char> &key, const void *p, size_t b) {
  const char *c = static_cast<const char *>(p);
  key.insert(key.end(), c, c + b);
}
std::vector<char> kp_key(const tn::KeepParams &kp) {
  std::vector<char> key;
  key_put(key, &kp.tau_rel, 8); key_put(key, &kp.tau_deg, 8); key_put(key, &kp.floor, 8);
  key_put(key, &kp.residual_tol, 8); key_put(key, &kp.model, sizeof(kp.model)); key_put(key, &kp.hx, sizeof(kp.hx));
  key_put(key, &kp.hy, sizeof(kp.hy)); key_put(key, &kp.hcount, sizeof(kp.hcount)); key_put(key, &kp.hcap, 8);
  key_put(key, &kp.split, 4); key_put(key, &kp.split_all, 4); key_put(key, kp.gemm_cfg, 12);
  key_put(key, &kp.tridiag_ql, 4);
  return key;
}

constexpr size_t kMaxGraphsPerPlan = 16;

// Capture the launches `launch(cs)` makes on the private stream cs into an executable graph.
template <class F>
int capture(hipStream_t cs, F &&launch, hipGraphExec_t *out) {
  *out = nullptr;
  HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  const int rc = launch(cs);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs, &graph);
  if (rc != TN_OK) { if (graph) (void)hipGraphDestroy(graph); return rc; }
  if (ec != hipSuccess) return fail(TN_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
  const hipError_t ei = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) { *out = nullptr; return fail(TN_EDEVICE, std::string("graph instantiation: ") + hipGetErrorString(ei)); }
  return TN_OK;
}

// The persistent launch of a batch: its launch descriptors and its captured graphs, one set
// per host thread and device (handles used on distinct threads never share them). A graph
// holds the single interpreter launch, whose arguments are the descriptor buffer, the
// network count and the launch parameters; the descriptors are copied in before each
// launch, so one graph serves every batch of that size and those parameters. Kept until
// the thread ends (not freed: HIP may already be shut down at process exit).
struct BatchCtx {
  tn::NetDev *d_nd = nullptr;
  size_t cap = 0;
  hipStream_t cap_stream = nullptr;
  std::map<std::vector<char>, hipGraphExec_t> execs;
};
thread_local std::map<int, BatchCtx> g_batch;

// The op launches of a network that runs op by op, on stream st.
int launch_segments(tn_net net, DevPlan *dp, const tn::KeepParams &kp, hipStream_t st) {
  for (const Seg &sg : dp->segs) {
    if (sg.kind == 0) HIP_TRY(tn::launch_interp_range(net->d_nd, sg.first, sg.last, kp, st));
    else if (sg.kind == 1) {
      const int sp = tn::op_split(kp, dp->plan.ops[size_t(sg.first)].flags);
      const int sk = sp ? 0 : sg.stream_k;          // FP64 only: streamed, else split K (tiled path)
      const int kc = sp || sk ? 1 : sg.kchunks;
      const int blocks = sk ? sg.stream_blocks
                            : (kc > 1 ? int(std::min<int64_t>(tn::kGridBlocks, int64_t(sg.blocks) * kc)) : sg.blocks);
      HIP_TRY(tn::launch_gemm_grid(net->d_nd, sg.first, blocks, sp, sg.piped, net->d_split, sg.split_blocks, kc,
                                   net->d_kpart, sk, st));
    } else {
      HIP_TRY(tn::launch_rescale_grid(net->d_nd, sg.first, sg.blocks, net->d_part, st));
    }
  }
  return TN_OK;
}

// Run a network op by op: its launches are captured once into a HIP graph (per plan
// and launch parameters) and the graph is launched on st.
int run_stepwise(tn_net net, DevPlan *dp, const tn::NetDev &nd, const tn::KeepParams &kp, hipStream_t st) {
  if (!net->d_nd && hipMalloc(&net->d_nd, sizeof(tn::NetDev)) != hipSuccess)
    return fail(TN_ENOMEM, "descriptor allocation failed");
  if (!net->d_part && hipMalloc(&net->d_part, tn::kGridBlocks * sizeof(double)) != hipSuccess)
    return fail(TN_ENOMEM, "grid scratch allocation failed");
  if (kp.split) {                           // planes for the largest chip-wide GEMM of the plan
    int64_t need = 0;
    for (const Seg &sg : dp->segs)
      if (sg.kind == 1 && tn::op_split(kp, dp->plan.ops[size_t(sg.first)].flags))
        need = std::max(need, sg.split_bytes);
    if (need > net->split_cap) {
      HIP_TRY(hipStreamSynchronize(st));    // earlier launches may still read the old planes
      if (net->d_split) (void)hipFree(net->d_split);
      net->d_split = nullptr;
      net->split_cap = 0;
      if (hipMalloc(&net->d_split, size_t(need)) != hipSuccess)
        return fail(TN_ENOMEM, "split scratch allocation of " + std::to_string(need) + " bytes failed");
      net->split_cap = need;
    }
  }
  {                                         // split-K partial products of the plan's FP64 tiled GEMMs
    int64_t need = 0;
    for (const Seg &sg : dp->segs)
      if (sg.kind == 1 && !tn::op_split(kp, dp->plan.ops[size_t(sg.first)].flags)) need = std::max(need, sg.kpart);
    if (need > net->kpart_cap) {
      HIP_TRY(hipStreamSynchronize(st));    // earlier launches may still use the old buffer
      if (net->d_kpart) (void)hipFree(net->d_kpart);
      net->d_kpart = nullptr;
      net->kpart_cap = 0;
      if (hipMalloc(&net->d_kpart, size_t(need) * sizeof(double)) != hipSuccess)
        return fail(TN_ENOMEM, "split-K scratch allocation of " + std::to_string(need * 8) + " bytes failed");
      net->kpart_cap = need;
    }
  }
  HIP_TRY(hipMemcpyAsync(net->d_nd, &nd, sizeof(nd), hipMemcpyHostToDevice, st));
  std::vector<char> key = kp_key(kp);
  key_put(key, &net->d_split, sizeof(net->d_split));
  key_put(key, &net->d_kpart, sizeof(net->d_kpart));
  auto it = dp->gexecs.find(key);
  if (it == dp->gexecs.end()) {
    if (dp->gexecs.size() >= kMaxGraphsPerPlan) {   // bounded cache: earlier launches have completed
      HIP_TRY(hipStreamSynchronize(st));
      for (auto &kv : dp->gexecs) (void)hipGraphExecDestroy(kv.second);
      dp->gexecs.clear();
    }
    if (!net->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&net->cap_stream, hipStreamNonBlocking));
    hipGraphExec_t ge = nullptr;
    const int rc = capture(net->cap_stream, [&](hipStream_t cs) { return launch_segments(net, dp, kp, cs); }, &ge);
    if (rc != TN_OK) return rc;
    it = dp->gexecs.emplace(std::move(key), ge).first;
  }
  HIP_TRY(hipGraphLaunch(it->second, st));
  return TN_OK;
}

// Run a list of prepared networks: those that fit one workgroup's pass in one
// persistent interpreter launch (one workgroup each), then each larger network op
// run by op run (a captured graph) on the same stream.
int run_batch(const std::vector<tn_net> &nets, const std::vector<DevPlan *> &plans, const tn_options &o,
              const tn::KeepParams &kp, double *seconds, std::vector<tn::NetScalars> &sc_out) {
  hipStream_t st = reinterpret_cast<hipStream_t>(o.hip_stream);
  const size_t n = nets.size();
  std::vector<size_t> order;                 // persistent ones first
  for (size_t i = 0; i < n; ++i)
    if (plans[i]->segs.empty()) order.push_back(i);
  const size_t n_persist = order.size();
  for (size_t i = 0; i < n; ++i)
    if (!plans[i]->segs.empty()) order.push_back(i);
  std::vector<tn::NetDev> nd(n);
  tn::NetScalars init{};
  init.sign = 1;
  struct SyncOnError {                     // an early return waits for the work already queued
    hipStream_t st;                        // (declared after the host buffers it protects)
    bool done = false;
    ~SyncOnError() {
      if (!done) (void)hipStreamSynchronize(st);
    }
  } pending{st};
  for (size_t q = 0; q < n; ++q) {
    const size_t i = order[q];
    HIP_TRY(hipMemcpyAsync(nets[i]->d_sc, &init, sizeof(init), hipMemcpyHostToDevice, st));
    nd[q].ops = plans[i]->d_ops;
    nd[q].n_ops = int64_t(plans[i]->plan.ops.size());
    nd[q].tab = plans[i]->d_tab;
    nd[q].ws = nets[i]->d_ws;
    nd[q].cst = nets[i]->d_const;
    nd[q].sc = nets[i]->d_sc;
    nd[q].dyn = reinterpret_cast<int32_t *>(nets[i]->d_ws + plans[i]->plan.dyn_off);
  }
  hipGraphExec_t persist = nullptr;
  const bool parts = o.chunks > 1 && n_persist > 0;
  if (n_persist > 0) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    BatchCtx &bc = g_batch[dev];
    if (bc.cap < n_persist) {               // grow: graphs refer to the old buffer
      HIP_TRY(hipStreamSynchronize(st));
      for (auto &kv : bc.execs) (void)hipGraphExecDestroy(kv.second);
      bc.execs.clear();
      if (bc.d_nd) (void)hipFree(bc.d_nd);
      bc.d_nd = nullptr;
      bc.cap = 0;
      const size_t cap = std::max<size_t>(n_persist, 64);
      if (hipMalloc(&bc.d_nd, cap * sizeof(tn::NetDev)) != hipSuccess)
        return fail(TN_ENOMEM, "launch descriptor allocation failed");
      bc.cap = cap;
    }
    std::vector<char> key = kp_key(kp);
    const int np = int(n_persist);
    key_put(key, &np, sizeof(np));
    auto it = bc.execs.find(key);
    if (parts) {
      // chunked: eager launches over parts of every op list (no graph)
    } else if (it == bc.execs.end()) {
      if (bc.execs.size() >= kMaxGraphsPerPlan) {
        HIP_TRY(hipStreamSynchronize(st));
        for (auto &kv : bc.execs) (void)hipGraphExecDestroy(kv.second);
        bc.execs.clear();
      }
      if (!bc.cap_stream) HIP_TRY(hipStreamCreateWithFlags(&bc.cap_stream, hipStreamNonBlocking));
      hipGraphExec_t ge = nullptr;
      tn::NetDev *d_nd = bc.d_nd;
      const int rc = capture(bc.cap_stream, [&](hipStream_t cs) -> int {
        HIP_TRY(tn::launch_interp(d_nd, np, kp, cs));
        return TN_OK;
      }, &ge);
      if (rc != TN_OK) return rc;
      it = bc.execs.emplace(std::move(key), ge).first;
    }
    if (!parts) {
      persist = it->second;
      HIP_TRY(hipMemcpyAsync(bc.d_nd, nd.data(), n_persist * sizeof(tn::NetDev), hipMemcpyHostToDevice, st));
    }
  }
  struct Events {                          // released on every return path
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Events() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } ev;
  HIP_TRY(hipEventCreate(&ev.e0));
  HIP_TRY(hipEventCreate(&ev.e1));
  HIP_TRY(hipEventRecord(ev.e0, st));
  if (persist) HIP_TRY(hipGraphLaunch(persist, st));
  if (parts) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    tn::NetDev *d_nd = g_batch[dev].d_nd;
    std::vector<tn::NetDev> part(nd.begin(), nd.begin() + long(n_persist));
    for (int32_t c = 0; c < o.chunks; ++c) {
      for (size_t q = 0; q < n_persist; ++q) {
        part[q].op_begin = nd[q].n_ops * c / o.chunks;
        part[q].op_end = nd[q].n_ops * (c + 1) / o.chunks;
      }
      HIP_TRY(hipMemcpyAsync(d_nd, part.data(), n_persist * sizeof(tn::NetDev), hipMemcpyHostToDevice, st));
      HIP_TRY(tn::launch_interp_parts(d_nd, int(n_persist), kp, st));
      HIP_TRY(hipStreamSynchronize(st));   // the next part's descriptors overwrite these
      if (o.progress) o.progress(o.progress_ctx, c + 1, o.chunks);
    }
  }
  for (size_t q = n_persist; q < n; ++q) {
    const int rc = run_stepwise(nets[order[q]], plans[order[q]], nd[q], kp, st);
    if (rc != TN_OK) return rc;
  }
  HIP_TRY(hipEventRecord(ev.e1, st));
  HIP_TRY(hipEventSynchronize(ev.e1));
  pending.done = true;
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, ev.e0, ev.e1));
  *seconds = ms * 1e-3;
  sc_out.resize(n);
  for (size_t i = 0; i < n; ++i)
    HIP_TRY(hipMemcpy(&sc_out[i], nets[i]->d_sc, sizeof(tn::NetScalars), hipMemcpyDeviceToHost));
  return TN_OK;
}

}  // namespace

extern "C" {

const char *tn_error_string(int status) {
  switch (status) {
    case TN_OK: return "ok";
    case TN_EINVAL: return "invalid argument";
    case TN_ENOMEM: return "out of memory";
    case TN_EDEVICE: return "device error";
    case TN_ENUMERIC: return "non-finite input";
    case TN_EUNSUPPORTED: return "unsupported by this build";
    default: return "unknown status";
  }
}

const char *tn_last_error(void) { return g_err.c_str(); }

int tn_create(const tn_tensor *tensors, int32_t n_tensors, const tn_edge *edges, int32_t n_edges, tn_net *out) {
  g_err.clear();
  if (!out) return fail(TN_EINVAL, "out is null");
  *out = nullptr;
  if (!tensors || n_tensors < 1) return fail(TN_EINVAL, "no tensors");
  if (n_edges > 0 && !edges) return fail(TN_EINVAL, "edges is null");
  std::vector<const int64_t *> dims(n_tensors);
  std::vector<int32_t> orders(n_tensors);
  for (int32_t t = 0; t < n_tensors; ++t) {
    orders[t] = tensors[t].order;
    dims[t] = tensors[t].dims;
    if (tensors[t].order > 0 && !tensors[t].dims) return fail(TN_EINVAL, "tensor dims is null");
    if (!tensors[t].data) return fail(TN_EINVAL, "tensor data is null");
  }
  std::vector<int32_t> e4(4 * size_t(std::max(n_edges, 0)));
  for (int32_t e = 0; e < n_edges; ++e) {
    e4[4 * e] = edges[e].t0; e4[4 * e + 1] = edges[e].m0; e4[4 * e + 2] = edges[e].t1; e4[4 * e + 3] = edges[e].m1;
  }
  auto net = std::make_unique<tn_net_s>();
  std::string err = tn::build_graph(dims.data(), orders.data(), n_tensors, e4.data(), n_edges, net->g);
  if (!err.empty()) return fail(TN_EINVAL, err);
  std::vector<double> host(std::max<int64_t>(net->g.const_size, 1), 0.0);
  for (int32_t t = 0; t < n_tensors; ++t) {
    int64_t size = 1;
    for (int64_t d : net->g.dims[t]) size *= d;
    for (int64_t i = 0; i < size; ++i) {
      double v = tensors[t].data[i];
      if (!std::isfinite(v)) return fail(TN_ENUMERIC, "tensor " + std::to_string(t) + " holds a non-finite value");
      host[net->g.const_off[t] + i] = v;
    }
  }
  int rc = check_device();
  if (rc != TN_OK) return rc;
  if (hipMalloc(&net->d_const, host.size() * 8) != hipSuccess) return fail(TN_ENOMEM, "constant area allocation failed");
  if (hipMalloc(&net->d_sc, sizeof(tn::NetScalars)) != hipSuccess) return fail(TN_ENOMEM, "scalar allocation failed");
  HIP_TRY(hipMemcpy(net->d_const, host.data(), host.size() * 8, hipMemcpyHostToDevice));
  *out = net.release();
  return TN_OK;
}

void tn_destroy(tn_net net) { delete net; }

static int contract_batch(const tn_net *nets, const tn_path *paths, const int32_t *max_ranks,
                          const int32_t *env_sizes, int32_t n, const tn_options &o, const tn::KeepParams &kp,
                          tn_result *outs);

// Options (NULL: defaults) checked and turned into the kernels' launch parameters.
static int prepare_options(const tn_options *opt, tn_options &o, tn::KeepParams &kp_out) {
  o = opt ? *opt : defaults();
  if (o.precision < TN_FP64 || o.precision > TN_SPLIT_FP16X3_ALL) return fail(TN_EINVAL, "unknown precision");
  if (o.eig != TN_EIG_EXACT && o.eig != TN_EIG_LEARNED) return fail(TN_EINVAL, "unknown eigensolve mode");
  if (o.eig == TN_EIG_LEARNED && !o.model) return fail(TN_EINVAL, "learned eigensolve needs a model");
  if (o.eig == TN_EIG_LEARNED && !(o.residual_tol > 0)) return fail(TN_EINVAL, "residual_tol must be > 0");
  if (o.chunks < 0) return fail(TN_EINVAL, "chunks must be >= 0");
  if (!(o.tau_rel >= 0) || !(o.tau_deg >= 0)) return fail(TN_EINVAL, "tau_rel and tau_deg must be >= 0");
  for (int c = 0; c < 3; ++c)
    if (o.gemm_config[c] < 0 || o.gemm_config[c] > tn::kGemmConfigs) return fail(TN_EINVAL, "gemm_config out of range");
  if (o.tridiag != TN_TRIDIAG_AUTO && o.tridiag != TN_TRIDIAG_QL) return fail(TN_EINVAL, "unknown tridiagonal solver");
  tn::KeepParams kp{o.tau_rel, o.tau_deg, tn::kClusterFloor * o.tau_rel};
  kp.tridiag_ql = o.tridiag == TN_TRIDIAG_QL;
  kp.residual_tol = o.residual_tol;
  kp.split = o.precision == TN_FP64 ? 0 : (o.precision == TN_SPLIT_BF16X3 || o.precision == TN_SPLIT_BF16X3_ALL ? 1 : 2);
  kp.split_all = o.precision == TN_SPLIT_BF16X3_ALL || o.precision == TN_SPLIT_FP16X3_ALL ? 1 : 0;
  for (int c = 0; c < 3; ++c) kp.gemm_cfg[c] = o.gemm_config[c];
  if (o.eig == TN_EIG_LEARNED) kp.model = o.model->d_w;
  kp_out = kp;
  return TN_OK;
}

int tn_contract_approx_batch(const tn_net *nets, const tn_path *paths, const int32_t *max_ranks,
                             const int32_t *env_sizes, int32_t n, const tn_options *opt, tn_result *outs) {
  g_err.clear();
  if (!nets || !paths || !outs || !max_ranks || !env_sizes || n < 1) return fail(TN_EINVAL, "null arrays or empty batch");
  for (int32_t i = 0; i < n; ++i) {
    if (max_ranks[i] < 1) return fail(TN_EINVAL, "max_rank must be >= 1");
    if (env_sizes[i] < 1) return fail(TN_EINVAL, "env_size must be >= 1");
  }
  tn_options o;
  tn::KeepParams kp{};
  const int rc = prepare_options(opt, o, kp);
  if (rc != TN_OK) return rc;
  return contract_batch(nets, paths, max_ranks, env_sizes, n, o, kp, outs);
}

static void fill_result(const tn::NetScalars &sc, const DevPlan &dp, double secs, tn_result &r) {
  std::memset(&r, 0, sizeof(r));
  if (sc.zero) {
    r.log_abs = -std::numeric_limits<double>::infinity();
    r.sign = 0;
  } else {
    r.log_abs = double(sc.exp_sum) * std::log(2.0) + sc.log_sum;
    r.sign = int32_t(sc.sign);
  }
  r.seconds = secs;
  r.flops = sc.flops;
  r.eig_flops = sc.eig_flops;
  r.n_eig = dp.plan.n_eig;
  r.n_fallback = sc.n_fallback;
  r.max_residual = sc.max_resid;
  r.n_learned = sc.n_learned;
  r.split_flops = sc.split_flops;
}

static int contract_batch(const tn_net *nets, const tn_path *paths, const int32_t *max_ranks,
                          const int32_t *env_sizes, int32_t n, const tn_options &o, const tn::KeepParams &kp,
                          tn_result *outs) {
  std::vector<tn_net> v(nets, nets + n);
  std::vector<DevPlan *> plans(n);
  for (int32_t i = 0; i < n; ++i) {
    if (!v[i]) return fail(TN_EINVAL, "null network handle");
    for (int32_t j = 0; j < i; ++j)
      if (v[j] == v[i]) return fail(TN_EINVAL, "a handle appears twice in one batch");
    std::vector<std::vector<int32_t>> slices;
    int rc = read_path(&paths[i], v[i]->g.nt, slices);
    if (rc != TN_OK) return rc;
    rc = get_plan(v[i], slices, max_ranks[i], env_sizes[i], &plans[i]);
    if (rc != TN_OK) return rc;
    rc = ensure_ws(v[i], plans[i]->plan.ws_size);
    if (rc != TN_OK) return rc;
  }
  double secs = 0;
  std::vector<tn::NetScalars> sc;
  int rc = run_batch(v, plans, o, kp, &secs, sc);
  if (rc != TN_OK) return rc;
  for (int32_t i = 0; i < n; ++i) {
    v[i]->last = sc[i];
    fill_result(sc[i], *plans[i], secs, outs[i]);
  }
  return TN_OK;
}

int tn_contract_approx(tn_net net, const tn_path *path, int32_t max_rank, int32_t env_size,
                       const tn_options *opt, tn_result *out) {
  return tn_contract_approx_batch(&net, path, &max_rank, &env_size, 1, opt, out);
}

int tn_contract_approx_noalloc(tn_net net, const tn_path *path, int32_t max_rank, int32_t env_size,
                               const tn_options *opt, tn_result *out) {
  g_err.clear();
  if (!net || !out) return fail(TN_EINVAL, "null network handle or result");
  if (max_rank < 1) return fail(TN_EINVAL, "max_rank must be >= 1");
  if (env_size < 1) return fail(TN_EINVAL, "env_size must be >= 1");
  tn_options o;
  tn::KeepParams kp{};
  int rc = prepare_options(opt, o, kp);
  if (rc != TN_OK) return rc;
  std::vector<std::vector<int32_t>> slices;
  rc = read_path(path, net->g.nt, slices);
  if (rc != TN_OK) return rc;
  DevPlan *dp = nullptr;
  rc = get_plan(net, slices, max_rank, env_size, &dp, /*device=*/false);
  if (rc != TN_OK) return rc;
  if (!dp->segs.empty())
    return fail(TN_EUNSUPPORTED, "the allocation-free entry point runs networks that fit one workgroup's pass; "
                                 "this plan has contractions that run over the whole chip");
  // scratch layout: descriptor | op list | index tables | workspace, each 256-byte aligned
  auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  const int64_t ob = int64_t(dp->plan.ops.size() * sizeof(tn::Op));
  const int64_t tb = int64_t(dp->plan.tables.size()) * 4;
  const int64_t wb = std::max<int64_t>(dp->plan.ws_size, 32) * 8;
  const int64_t off_ops = up(sizeof(tn::NetDev)), off_tab = off_ops + up(ob), off_ws = off_tab + up(tb);
  const int64_t total = off_ws + wb;
  if (total > tn::kNoAllocScratchBytes)
    return fail(TN_EUNSUPPORTED, "the plan needs " + std::to_string(total) + " bytes of device scratch; the "
                                 "allocation-free entry point holds " + std::to_string(tn::kNoAllocScratchBytes));
  char *base = nullptr;
  HIP_TRY(tn::noalloc_scratch(&base));
  double *ws = reinterpret_cast<double *>(base + off_ws);
  tn::NetDev nd{reinterpret_cast<const tn::Op *>(base + off_ops), int64_t(dp->plan.ops.size()),
                reinterpret_cast<const int32_t *>(base + off_tab), ws, net->d_const, net->d_sc,
                reinterpret_cast<int32_t *>(ws + dp->plan.dyn_off)};
  tn::NetScalars init{};
  init.sign = 1;
  hipStream_t st = reinterpret_cast<hipStream_t>(o.hip_stream);
  // the workspace is not cleared: every op writes what a later op reads
  if (ob) HIP_TRY(hipMemcpyAsync(base + off_ops, dp->plan.ops.data(), size_t(ob), hipMemcpyHostToDevice, st));
  if (tb) HIP_TRY(hipMemcpyAsync(base + off_tab, dp->plan.tables.data(), size_t(tb), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(base, &nd, sizeof(nd), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(net->d_sc, &init, sizeof(init), hipMemcpyHostToDevice, st));
  const auto t0 = std::chrono::steady_clock::now();
  HIP_TRY(tn::launch_interp(reinterpret_cast<const tn::NetDev *>(base), 1, kp, st));
  HIP_TRY(hipStreamSynchronize(st));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  tn::NetScalars sc{};
  HIP_TRY(hipMemcpy(&sc, net->d_sc, sizeof(sc), hipMemcpyDeviceToHost));
  net->last = sc;
  fill_result(sc, *dp, secs, *out);
  return TN_OK;
}

int tn_plan_json(const int64_t *dims_flat, const int32_t *orders, int32_t n_tensors, const tn_edge *edges,
                 int32_t n_edges, const tn_path *path, int32_t env_size, char *buf, int64_t *len) {
  g_err.clear();
  if (!orders || !len || n_tensors < 1) return fail(TN_EINVAL, "null arguments");
  std::vector<const int64_t *> dims(n_tensors);
  int64_t off = 0;
  for (int32_t t = 0; t < n_tensors; ++t) {
    dims[t] = dims_flat + off;
    off += std::max(orders[t], 0);
  }
  std::vector<int32_t> e4(4 * size_t(std::max(n_edges, 0)));
  for (int32_t e = 0; e < n_edges; ++e) {
    e4[4 * e] = edges[e].t0; e4[4 * e + 1] = edges[e].m0; e4[4 * e + 2] = edges[e].t1; e4[4 * e + 3] = edges[e].m1;
  }
  tn::Graph g;
  std::string err = tn::build_graph(dims.data(), orders, n_tensors, e4.data(), n_edges, g);
  if (!err.empty()) return fail(TN_EINVAL, err);
  std::vector<std::vector<int32_t>> slices;
  int rc = read_path(path, n_tensors, slices);
  if (rc != TN_OK) return rc;
  tn::PlanArgs pa;
  pa.slices = slices;
  pa.chi = 1;
  pa.env = env_size;
  tn::Plan plan;
  bool unsup = false;
  err = tn::make_plan(g, pa, plan, &unsup);
  if (!err.empty()) return fail(unsup ? TN_EUNSUPPORTED : TN_EINVAL, err);
  int64_t need = int64_t(plan.plan_json.size()) + 1;
  if (buf && *len >= need) std::memcpy(buf, plan.plan_json.c_str(), size_t(need));
  int64_t have = *len;
  *len = need;
  if (buf && have < need) return fail(TN_EINVAL, "buffer too small");
  return TN_OK;
}

// ---------------------------------------------------------------- learned warm start

static uint64_t host_splitmix64(uint64_t &state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int tn_model_create(uint64_t seed, tn_model *out) {
  g_err.clear();
  if (!out) return fail(TN_EINVAL, "out is null");
  *out = nullptr;
  int rc = check_device();
  if (rc != TN_OK) return rc;
  const int P = tn::kMlpParams;
  std::vector<float> w(P, 0.0f);
  uint64_t st = seed;
  auto uni = [&](double lim) { return float((double(host_splitmix64(st) >> 11) * 0x1.0p-53 * 2.0 - 1.0) * lim); };
  int o = 0;
  const int shapes[3][2] = {{8, 32}, {32, 32}, {32, 1}};
  for (auto &sh : shapes) {                 // Glorot-uniform weights, zero biases
    const double lim = std::sqrt(6.0 / (sh[0] + sh[1]));
    for (int i = 0; i < sh[0] * sh[1]; ++i) w[o++] = uni(lim);
    o += sh[1];
  }
  auto m = std::make_unique<tn_model_s>();
  if (hipMalloc(&m->d_w, P * 4) != hipSuccess || hipMalloc(&m->d_m, P * 4) != hipSuccess ||
      hipMalloc(&m->d_v, P * 4) != hipSuccess || hipMalloc(&m->d_loss, 16) != hipSuccess)
    return fail(TN_ENOMEM, "model allocation failed");
  std::vector<float> zero(P, 0.0f);
  HIP_TRY(hipMemcpy(m->d_w, w.data(), P * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(m->d_m, zero.data(), P * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(m->d_v, zero.data(), P * 4, hipMemcpyHostToDevice));
  *out = m.release();
  return TN_OK;
}

int tn_model_set(tn_model m, const float *w, int64_t n) {
  g_err.clear();
  if (!m || !w || n != tn::kMlpParams) return fail(TN_EINVAL, "expected 1377 weights");
  HIP_TRY(hipMemcpy(m->d_w, w, n * 4, hipMemcpyHostToDevice));
  return TN_OK;
}

int tn_model_get(tn_model m, float *w, int64_t n) {
  g_err.clear();
  if (!m || !w || n != tn::kMlpParams) return fail(TN_EINVAL, "expected 1377 weights");
  HIP_TRY(hipMemcpy(w, m->d_w, n * 4, hipMemcpyDeviceToHost));
  return TN_OK;
}

int tn_model_grad(tn_model m, const float *X, const float *y, int32_t rows, float *grad, double *loss) {
  g_err.clear();
  if (!m || !X || !y || !grad || rows < 1 || rows > tn::kMlpBatch) return fail(TN_EINVAL, "1..128 rows expected");
  float *dx = nullptr, *dy = nullptr, *dg = nullptr;
  if (hipMalloc(&dx, rows * 8 * 4) != hipSuccess || hipMalloc(&dy, rows * 4) != hipSuccess ||
      hipMalloc(&dg, tn::kMlpParams * 4) != hipSuccess) {
    (void)hipFree(dx); (void)hipFree(dy); (void)hipFree(dg);
    return fail(TN_ENOMEM, "gradient buffers");
  }
  hipError_t e = hipMemcpy(dx, X, rows * 8 * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dy, y, rows * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = tn::launch_mlp_train(m->d_w, m->d_m, m->d_v, dx, dy, rows, 1, rows, 0.0f, 0, 0, m->d_loss, dg, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  float l = 0.0f;
  if (e == hipSuccess) e = hipMemcpy(grad, dg, tn::kMlpParams * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&l, m->d_loss, 4, hipMemcpyDeviceToHost);
  (void)hipFree(dx); (void)hipFree(dy); (void)hipFree(dg);
  if (e != hipSuccess) return fail(TN_EDEVICE, std::string("gradient: ") + hipGetErrorString(e));
  if (loss) *loss = l;
  return TN_OK;
}

int tn_model_train(tn_model m, tn_dataset ds, int32_t steps, int32_t batch, double lr, uint64_t seed,
                   double *final_loss) {
  g_err.clear();
  if (!m || !ds || steps < 1 || batch < 1 || batch > tn::kMlpBatch || !(lr > 0)) return fail(TN_EINVAL, "bad training arguments");
  int cnt = 0;
  HIP_TRY(hipMemcpy(&cnt, ds->d_count, 4, hipMemcpyDeviceToHost));
  const int64_t rows = std::min<int64_t>(cnt, ds->cap);
  if (rows < 1) return fail(TN_EINVAL, "empty dataset");
  HIP_TRY(tn::launch_mlp_train(m->d_w, m->d_m, m->d_v, ds->d_x, ds->d_y, rows, steps, batch, float(lr), seed, m->t,
                               m->d_loss, nullptr, nullptr));
  HIP_TRY(hipDeviceSynchronize());
  m->t += steps;
  float l = 0.0f;
  HIP_TRY(hipMemcpy(&l, m->d_loss, 4, hipMemcpyDeviceToHost));
  if (final_loss) *final_loss = l;
  return TN_OK;
}

void tn_model_destroy(tn_model m) { delete m; }

int tn_dataset_create(int64_t capacity_rows, tn_dataset *out) {
  g_err.clear();
  if (!out || capacity_rows < 1) return fail(TN_EINVAL, "capacity must be >= 1");
  *out = nullptr;
  int rc = check_device();
  if (rc != TN_OK) return rc;
  auto d = std::make_unique<tn_dataset_s>();
  d->cap = capacity_rows;
  if (hipMalloc(&d->d_x, capacity_rows * 8 * 4) != hipSuccess || hipMalloc(&d->d_y, capacity_rows * 4) != hipSuccess ||
      hipMalloc(&d->d_count, 4) != hipSuccess)
    return fail(TN_ENOMEM, "dataset allocation failed");
  int zero = 0;
  HIP_TRY(hipMemcpy(d->d_count, &zero, 4, hipMemcpyHostToDevice));
  *out = d.release();
  return TN_OK;
}

int tn_dataset_size(tn_dataset ds, int64_t *rows) {
  g_err.clear();
  if (!ds || !rows) return fail(TN_EINVAL, "null arguments");
  int cnt = 0;
  HIP_TRY(hipMemcpy(&cnt, ds->d_count, 4, hipMemcpyDeviceToHost));
  *rows = std::min<int64_t>(cnt, ds->cap);
  return TN_OK;
}

int tn_dataset_read(tn_dataset ds, float *X, float *y, int64_t rows) {
  g_err.clear();
  if (!ds || !X || !y || rows < 0 || rows > ds->cap) return fail(TN_EINVAL, "bad read");
  if (rows == 0) return TN_OK;
  HIP_TRY(hipMemcpy(X, ds->d_x, rows * 8 * 4, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(y, ds->d_y, rows * 4, hipMemcpyDeviceToHost));
  return TN_OK;
}

void tn_dataset_destroy(tn_dataset ds) { delete ds; }

int tn_harvest(tn_net net, const tn_path *path, int32_t max_rank, int32_t env_size, tn_dataset ds, tn_result *out) {
  g_err.clear();
  if (!net || !ds || !out) return fail(TN_EINVAL, "null arguments");
  if (max_rank < 1 || env_size < 1) return fail(TN_EINVAL, "max_rank and env_size must be >= 1");
  tn_options o = defaults();
  tn::KeepParams kp{o.tau_rel, o.tau_deg, tn::kClusterFloor * o.tau_rel};
  kp.hx = ds->d_x;
  kp.hy = ds->d_y;
  kp.hcount = ds->d_count;
  kp.hcap = ds->cap;
  return contract_batch(&net, path, &max_rank, &env_size, 1, o, kp, out);
}

// ---------------------------------------------------------------- diagnostics

int tn_plan_stats(tn_net net, const tn_path *path, int32_t max_rank, int32_t env_size, int64_t *stats) {
  g_err.clear();
  if (!net || !stats) return fail(TN_EINVAL, "null arguments");
  std::vector<std::vector<int32_t>> slices;
  int rc = read_path(path, net->g.nt, slices);
  if (rc != TN_OK) return rc;
  DevPlan *dp = nullptr;
  rc = get_plan(net, slices, max_rank, env_size, &dp);
  if (rc != TN_OK) return rc;
  stats[0] = int64_t(dp->plan.ops.size());
  stats[1] = int64_t(dp->plan.tables.size());
  stats[2] = dp->plan.ws_size;
  stats[3] = dp->plan.flops;
  stats[4] = dp->plan.eig_flops;
  stats[5] = dp->plan.n_eig;
  stats[6] = dp->plan.max_eig_dim;
  int64_t grid_ops = 0;
  for (const Seg &sg : dp->segs) grid_ops += sg.kind != 0 ? 1 : 0;
  stats[7] = grid_ops;
  stats[8] = dp->plan.n_qr;
  return TN_OK;
}

int tn_profile_last(tn_net net, double *seconds_by_kind) {
  g_err.clear();
  if (!net || !seconds_by_kind) return fail(TN_EINVAL, "null arguments");
  int dev = 0, khz = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  for (int k = 0; k < 8; ++k) seconds_by_kind[k] = khz > 0 ? double(net->last.ticks[k]) / (double(khz) * 1e3) : 0.0;
  seconds_by_kind[8] = double(net->last.n_rot);   // QL rotations of the last contraction
  for (int r = 0; r < 4; ++r) seconds_by_kind[9 + r] = double(net->last.rej[r]);
  for (int r = 0; r < 4; ++r)
    seconds_by_kind[13 + r] = khz > 0 ? double(net->last.lticks[r]) / (double(khz) * 1e3) : 0.0;
  seconds_by_kind[17] = khz > 0 ? double(net->last.qr_ticks) / (double(khz) * 1e3) : 0.0;
  return TN_OK;
}

// Run single device ops on host data through the same interpreter (kernel tests).
// slots: the kept-rank slots (in: initial extents, default 1; out: as left by the ops).
static int run_single(const std::vector<tn::Op> &ops, const std::vector<int32_t> &tab, std::vector<double> &ws,
                      const std::vector<double> &cst, const tn::KeepParams &kp, tn::NetScalars *sc_out,
                      std::vector<int32_t> *slots_io = nullptr, int grid_blocks = 0, bool grid_piped = false,
                      int grid_kchunks = 1, int grid_stream_k = 0) {
  int rc = check_device();
  if (rc != TN_OK) return rc;
  tn::Op *d_ops = nullptr;
  int32_t *d_tab = nullptr;
  double *d_ws = nullptr, *d_cst = nullptr;
  tn::NetScalars *d_sc = nullptr;
  tn::NetDev *d_nd = nullptr;
  unsigned short *d_planes = nullptr;
  double *d_kpart = nullptr;
  auto cleanup = [&]() {
    (void)hipFree(d_ops); (void)hipFree(d_tab); (void)hipFree(d_ws); (void)hipFree(d_cst);
    (void)hipFree(d_sc); (void)hipFree(d_nd); (void)hipFree(d_planes); (void)hipFree(d_kpart);
  };
  if (hipMalloc(&d_ops, ops.size() * sizeof(tn::Op)) != hipSuccess ||
      hipMalloc(&d_tab, std::max<size_t>(tab.size(), 1) * 4) != hipSuccess ||
      hipMalloc(&d_ws, (ws.size() + 32) * 8) != hipSuccess ||
      hipMalloc(&d_cst, std::max<size_t>(cst.size(), 1) * 8) != hipSuccess ||
      hipMalloc(&d_sc, sizeof(tn::NetScalars)) != hipSuccess ||
      hipMalloc(&d_nd, sizeof(tn::NetDev)) != hipSuccess) {
    cleanup();
    return fail(TN_ENOMEM, "diagnostic allocation failed");
  }
  tn::NetScalars init{};
  init.sign = 1;
  // the first 32 doubles of the diagnostic workspace hold the kept-rank slots
  tn::NetDev nd{d_ops, int64_t(ops.size()), d_tab, d_ws + 32, d_cst, d_sc, reinterpret_cast<int32_t *>(d_ws)};
  hipError_t e = hipMemcpy(d_ops, ops.data(), ops.size() * sizeof(tn::Op), hipMemcpyHostToDevice);
  if (e == hipSuccess && !tab.empty()) e = hipMemcpy(d_tab, tab.data(), tab.size() * 4, hipMemcpyHostToDevice);
  std::vector<int32_t> slots(64, 1);
  if (slots_io)
    for (size_t i = 0; i < slots_io->size() && i < slots.size(); ++i) slots[i] = (*slots_io)[i];
  if (e == hipSuccess) e = hipMemcpy(d_ws, slots.data(), 64 * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess && !ws.empty()) e = hipMemcpy(d_ws + 32, ws.data(), ws.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess && !cst.empty()) e = hipMemcpy(d_cst, cst.data(), cst.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_sc, &init, sizeof(init), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_nd, &nd, sizeof(nd), hipMemcpyHostToDevice);
  int split_blocks = 0;
  if (e == hipSuccess && grid_blocks > 0 && kp.split) {
    const tn::Op &op = ops[0];
    split_blocks = tn::split_grid_blocks(op.am.n, op.bn.n, op.K);
    e = hipMalloc(&d_planes, size_t(tn::split_scratch_bytes(op.am.n, op.bn.n, op.K)));
  }
  const int kc = grid_blocks > 0 && !kp.split && !grid_piped && !grid_stream_k ? grid_kchunks : 1;
  if (e == hipSuccess && kc > 1) {
    const tn::Op &op = ops[0];
    e = hipMalloc(&d_kpart, size_t(kc) * op.am.n * op.bn.n * sizeof(double));
  }
  if (e == hipSuccess)   // one op over the whole chip, else the interpreter's single workgroup
    e = grid_blocks > 0 ? tn::launch_gemm_grid(d_nd, 0, kc > 1 ? std::min(tn::kGridBlocks, grid_blocks * kc) : grid_blocks,
                                               kp.split, grid_piped, d_planes, split_blocks, kc, d_kpart,
                                               grid_stream_k, nullptr)
                        : tn::launch_interp(d_nd, 1, kp, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess && !ws.empty()) e = hipMemcpy(ws.data(), d_ws + 32, ws.size() * 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess && sc_out) e = hipMemcpy(sc_out, d_sc, sizeof(tn::NetScalars), hipMemcpyDeviceToHost);
  if (e == hipSuccess && slots_io) {
    e = hipMemcpy(slots.data(), d_ws, 64 * 4, hipMemcpyDeviceToHost);
    *slots_io = slots;
  }
  cleanup();
  if (e != hipSuccess) return fail(TN_EDEVICE, std::string("diagnostic run: ") + hipGetErrorString(e));
  return TN_OK;
}

int tn_debug_gemm(const double *A, int64_t sam, int64_t sak, const double *B, int64_t sbk, int64_t sbn,
                  double *C, int32_t M, int32_t N, int32_t K, int32_t lo_split, int32_t precision,
                  int32_t chip_wide) {
  g_err.clear();
  if (!A || !B || !C || M < 1 || N < 1 || K < 1) return fail(TN_EINVAL, "bad gemm arguments");
  if (precision < TN_FP64 || precision > TN_SPLIT_FP16X3) return fail(TN_EINVAL, "unknown precision");
  if (lo_split < 1) lo_split = 1;
  std::vector<int32_t> tab;
  auto push_map = [&](int32_t n, int64_t stride, tn::IdxMap &m) {
    int32_t lo = std::min(lo_split, n);
    int32_t nh = (n + lo - 1) / lo;
    m.hi = int64_t(tab.size());
    for (int32_t h = 0; h < nh; ++h) tab.push_back(int32_t(int64_t(h) * lo * stride));
    m.lo = int64_t(tab.size());
    for (int32_t l = 0; l < lo; ++l) tab.push_back(int32_t(l * stride));
    m.lo_n = lo;
    m.n = n;
  };
  int64_t maxa = (M - 1) * sam + (K - 1) * sak + 1, maxb = (K - 1) * sbk + (N - 1) * sbn + 1;
  tn::Op op{};
  op.kind = tn::OP_GEMM;
  op.flags = tn::F_A_CONST | tn::F_B_CONST | (sak == 1 ? tn::F_A_KFAST : 0) | (sbn == 1 ? tn::F_B_NFAST : 0);
  push_map(M, sam, op.am);
  push_map(N, sbn, op.bn);
  op.K = K;
  op.bm = tn::Box{0, M, {0}, {0}};
  op.bnb = tn::Box{0, N, {0}, {0}};
  op.bk_ = tn::Box{0, K, {0}, {0}};
  op.ak = int32_t(tab.size());
  for (int32_t k = 0; k < K; ++k) tab.push_back(int32_t(k * sak));
  op.bk = int32_t(tab.size());
  for (int32_t k = 0; k < K; ++k) tab.push_back(int32_t(k * sbk));
  std::vector<double> cst(A, A + maxa);
  op.a = 0;
  op.b = (maxa + 31) / 32 * 32;
  cst.resize(op.b, 0.0);
  cst.insert(cst.end(), B, B + maxb);
  op.c = 0;
  std::vector<double> ws(int64_t(M) * N, 0.0);
  tn::KeepParams kp{kTauRel, kTauDeg, tn::kClusterFloor * kTauRel};
  if (precision < TN_FP64 || precision > TN_SPLIT_FP16X3_ALL) return fail(TN_EINVAL, "unknown precision");
  kp.split = precision == TN_FP64 ? 0 : (precision == TN_SPLIT_BF16X3 || precision == TN_SPLIT_BF16X3_ALL ? 1 : 2);
  kp.split_all = 1;                 // the diagnostic product is split whatever its class
  int blocks = 0, kchunks = 1, stream_k = 0;
  bool piped = false;
  if (chip_wide) {   // the launch the planner gives a chip-wide contraction of this shape
    blocks = int(std::min<int64_t>(tn::kGridBlocks, ((int64_t(M) + 63) / 64) * ((int64_t(N) + 63) / 64)));
    piped = int64_t(M) + K <= int64_t(tn::kGridOffsetDoubles) && int64_t(M) * N < (int64_t(1) << 31);
    if (!piped) kchunks = tn::grid_kchunks(M, N, K);
    if (!kp.split) stream_k = tn::stream_kclass(M, N, K);
    if (stream_k) blocks = tn::stream_blocks(N);
  }
  int rc = run_single({op}, tab, ws, cst, kp, nullptr, nullptr, blocks, piped, kchunks, stream_k);
  if (rc != TN_OK) return rc;
  std::memcpy(C, ws.data(), ws.size() * 8);
  return TN_OK;
}

int tn_debug_eig(const double *L, int32_t n, int32_t ucols, int32_t rest, const tn_options *opt, double *U,
                 int64_t *stats) {
  g_err.clear();
  if (!L || !U || n < 1 || n > tn::kMaxEigDim || ucols < 1 || ucols > n) return fail(TN_EINVAL, "bad eig arguments");
  if (rest < 0 || (rest > 0 && (n % rest != 0 || n / rest < 1))) return fail(TN_EINVAL, "rest must divide n");
  tn_options o = opt ? *opt : defaults();
  if (o.eig == TN_EIG_LEARNED && (!o.model || !(o.residual_tol > 0)))
    return fail(TN_EINVAL, "learned mode needs a model and residual_tol > 0");
  const int64_t np = n + (n & 1);
  tn::Op op{};
  op.kind = tn::OP_EIG;
  op.count = n;
  op.K = ucols;
  // rows are (bond, leaf) with the bond extent held in kept-rank slot 1, or plain rows
  op.bm = rest > 0 ? tn::Box{1, rest, {1}, {n / rest}} : tn::Box{0, n, {0}, {0}};
  op.out_dyn = 0;
  op.a = 0;
  int64_t lsz = (int64_t(n) * n + 31) / 32 * 32;
  op.c = lsz;
  int64_t usz = (int64_t(n) * ucols + 31) / 32 * 32;
  op.b = lsz + usz;
  op.flags |= tn::F_V_GLOBAL;
  std::vector<double> ws(lsz + usz + 3 * (np * np + np), 0.0);   // the scratch the planner gives
  std::memcpy(ws.data(), L, size_t(n) * n * 8);
  if (o.tridiag != TN_TRIDIAG_AUTO && o.tridiag != TN_TRIDIAG_QL) return fail(TN_EINVAL, "unknown tridiagonal solver");
  tn::KeepParams kp{o.tau_rel, o.tau_deg, tn::kClusterFloor * o.tau_rel};
  kp.tridiag_ql = o.tridiag == TN_TRIDIAG_QL;
  if (o.eig == TN_EIG_LEARNED) {
    kp.model = o.model->d_w;
    kp.residual_tol = o.residual_tol;
  }
  tn::NetScalars sc{};
  std::vector<int32_t> slots(2, 1);
  if (rest > 0) slots[1] = n / rest;
  int rc = run_single({op}, {}, ws, {}, kp, &sc, &slots);
  if (rc != TN_OK) return rc;
  const int32_t k = slots[0];
  for (int32_t i = 0; i < n; ++i)          // device layout U[j][i] -> host n x ucols, zero past k
    for (int32_t j = 0; j < ucols; ++j) U[int64_t(i) * ucols + j] = j < k ? ws[lsz + int64_t(j) * n + i] : 0.0;
  if (stats) {
    stats[0] = sc.n_fallback;
    stats[1] = sc.n_learned;
    stats[2] = k;
    for (int r = 0; r < 4; ++r) stats[3 + r] = sc.rej[r];
    stats[7] = 0;
  }
  return TN_OK;
}

int tn_debug_rescale(double *x, int64_t count, int64_t *exponent) {
  g_err.clear();
  if (!x || count < 1) return fail(TN_EINVAL, "bad rescale arguments");
  tn::Op op{};
  op.kind = tn::OP_RESCALE;
  op.flags = tn::F_ACCUM;
  op.c = 0;
  op.count = 1;
  op.bm = tn::Box{0, int32_t(count), {0}, {0}};
  op.bnb = tn::Box{0, 1, {0}, {0}};
  std::vector<double> ws(x, x + count);
  tn::KeepParams kp{kTauRel, kTauDeg, tn::kClusterFloor * kTauRel};
  tn::NetScalars sc{};
  int rc = run_single({op}, {}, ws, {}, kp, &sc);
  if (rc != TN_OK) return rc;
  std::memcpy(x, ws.data(), size_t(count) * 8);
  if (exponent) *exponent = sc.exp_sum;
  return TN_OK;
}

}  // extern "C"
