// Ensembles of independent 1+1 diamonds: plan, run, HIP-graph capture and the tile
// autotuner.  (The thesis averages its action measurements over ensembles of
// causal sets; here the ensemble is one pipeline of five launches.)
//
// Plan: per-instance offsets into three concatenated buffers (coordinates, matrices,
// histograms), the builder's work list (one item per 64x64 block pair bi <= bj) and
// the counters' work lists (one item per row panel I of output tiles, i.e. all tiles
// (I, J >= I) of an instance, so a workgroup keeps one instance's histogram in LDS for
// a whole panel), sorted by cost across all instances so the persistent counter
// balances instances of very different sizes.  These tables live in device memory owned by the plan, uploaded
// once at plan time, so a run only enqueues kernels: fill, sprinkle, build, count
// (one persistent launch per tile shape in use), action.
//
// Tile shape: the MFMA counter has 128x128 and 256x256 output tiles.  Instances with
// n >= tile256_min_n use the larger one.  cs_autotune measures the crossover on the
// device and stores it as JSON; cs_batch_plan reads that file when given its path.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "common.h"

using namespace cs;

struct cs_batch_plan_t {
  int64_t count = 0;
  int counter = CS_COUNT_MFMA;
  int n_eps = 0;
  std::vector<BatchInst> inst;
  int64_t coords_len = 0, bits_len = 0, hist_len = 0;
  int64_t n_build = 0;
  int64_t n_items[3] = {0, 0, 0};  // per mode slot: bitset(0), MFMA 128 (1), MFMA 256 (2)
  size_t ws_bytes = 0, off_coords = 0, off_bits = 0;
  void* dev = nullptr;              // device tables
  BatchInst* d_inst = nullptr;
  double* d_eps = nullptr;
  uint32_t* d_build = nullptr;
  uint32_t* d_items[3] = {nullptr, nullptr, nullptr};
  int device = 0;
};

namespace {

constexpr int kModeOf[3] = {0, 2, 4};
constexpr int64_t kDefaultTile256MinN = 4096;

int64_t read_tile256_min_n(const char* path) {
  if (!path || !*path) return kDefaultTile256MinN;
  FILE* f = fopen(path, "r");
  if (!f) return kDefaultTile256MinN;
  char buf[4096];
  size_t got = fread(buf, 1, sizeof(buf) - 1, f);
  fclose(f);
  buf[got] = 0;
  const char* key = strstr(buf, "\"tile256_min_n\"");
  if (!key) return kDefaultTile256MinN;
  const char* colon = strchr(key, ':');
  if (!colon) return kDefaultTile256MinN;
  long long v = atoll(colon + 1);
  return v > 0 ? (int64_t)v : kDefaultTile256MinN;
}

size_t take(size_t* off, size_t bytes) {
  size_t o = *off;
  *off = align_up(*off + bytes, 256);
  return o;
}

cs_status build_plan(int64_t count, const int64_t* n, int counter, int n_eps, const double* eps,
                     int64_t tile256_min_n, cs_batch_plan_t* p) {
  p->count = count;
  p->counter = counter;
  p->n_eps = n_eps;
  p->inst.resize(count);
  std::vector<uint32_t> build;
  struct Item {
    uint32_t packed;
    int64_t cost;
  };
  std::vector<Item> items[3];
  int64_t coff = 0, boff = 0, hoff = 0;
  for (int64_t k = 0; k < count; ++k) {
    BatchInst& d = p->inst[k];
    d.n = n[k];
    d.ld = ld_words(d.n);
    d.coord_off = coff;
    d.bits_off = boff;
    d.hist_off = hoff;
    coff += 2 * d.n;
    boff += d.n * d.ld;
    hoff += d.n - 1;
    const int64_t nb = ceil_div(d.n, 64);
    for (int64_t bi = 0; bi < nb; ++bi)
      for (int64_t bj = bi; bj < nb; ++bj)
        build.push_back((uint32_t)(k << 16 | bi << 8 | bj));
    int slot = counter == CS_COUNT_BITSET ? 0 : (d.n >= tile256_min_n ? 2 : 1);
    const int64_t BM = slot == 2 ? 256 : 128;
    const int64_t T = ceil_div(d.n, BM);
    for (int64_t I = 0; I < T; ++I)  // row panel I: tiles (I, J) for J = I .. T-1
      items[slot].push_back({(uint32_t)(k << 16 | I << 8), (T - I) * (T - I + 1) / 2 * BM * BM * BM});
  }
  p->coords_len = coff;
  p->bits_len = boff;
  p->hist_len = hoff;
  p->n_build = (int64_t)build.size();
  for (int s = 0; s < 3; ++s) {
    std::stable_sort(items[s].begin(), items[s].end(),
                     [](const Item& a, const Item& b) { return a.cost > b.cost; });
    p->n_items[s] = (int64_t)items[s].size();
  }

  // Caller workspace: [3 tile counters][coordinates][matrices].
  size_t off = 0;
  take(&off, 256);
  p->off_coords = take(&off, sizeof(double) * (size_t)coff);
  p->off_bits = take(&off, sizeof(uint64_t) * (size_t)boff);
  p->ws_bytes = off;

  // Device tables owned by the plan.
  size_t doff = 0;
  size_t o_inst = take(&doff, sizeof(BatchInst) * count);
  size_t o_eps = take(&doff, sizeof(double) * (n_eps > 0 ? n_eps : 1));
  size_t o_build = take(&doff, sizeof(uint32_t) * build.size());
  size_t o_items[3];
  for (int s = 0; s < 3; ++s) o_items[s] = take(&doff, sizeof(uint32_t) * items[s].size());
  CS_HIP_CHECK(hipGetDevice(&p->device));
  CS_HIP_CHECK(hipMalloc(&p->dev, doff));
  char* b = (char*)p->dev;
  p->d_inst = (BatchInst*)(b + o_inst);
  p->d_eps = (double*)(b + o_eps);
  p->d_build = (uint32_t*)(b + o_build);
  std::vector<char> host(doff, 0);
  memcpy(host.data() + o_inst, p->inst.data(), sizeof(BatchInst) * count);
  if (n_eps > 0) memcpy(host.data() + o_eps, eps, sizeof(double) * n_eps);
  memcpy(host.data() + o_build, build.data(), sizeof(uint32_t) * build.size());
  for (int s = 0; s < 3; ++s) {
    p->d_items[s] = (uint32_t*)(b + o_items[s]);
    uint32_t* dst = (uint32_t*)(host.data() + o_items[s]);
    for (size_t q = 0; q < items[s].size(); ++q) dst[q] = items[s][q].packed;
  }
  CS_HIP_CHECK(hipMemcpy(p->dev, host.data(), doff, hipMemcpyHostToDevice));
  return CS_OK;
}

cs_status run_counts(cs_batch_plan_t* p, const uint64_t* bits, uint64_t* hist, unsigned int* ctr,
                     hipStream_t st) {
  for (int s = 0; s < 3; ++s) {
    if (!p->n_items[s]) continue;
    cs_status r = launch_count_batch(kModeOf[s], p->counter == CS_COUNT_MFMA_FP4, bits, p->d_inst,
                                     p->d_items[s], p->n_items[s], hist, ctr + s, st);
    if (r != CS_OK) return r;
  }
  return CS_OK;
}

}  // namespace

extern "C" {

cs_status cs_batch_plan(int64_t count, const int64_t* n, int counter, int n_eps, const double* eps,
                        const char* tune_cache, cs_batch_plan_handle* plan) {
  if (!plan) return CS_ERR_INVALID_ARG;
  *plan = nullptr;
  if (counter != CS_COUNT_BITSET && counter != CS_COUNT_MFMA && counter != CS_COUNT_MFMA_FP4)
    return CS_ERR_UNSUPPORTED;
  if (count < 1 || count > 65535 || !n || n_eps < 0 || (n_eps > 0 && !eps))
    return CS_ERR_INVALID_ARG;
  for (int64_t k = 0; k < count; ++k)
    if (n[k] < 2 || n[k] > kBatchMaxN) return CS_ERR_INVALID_ARG;
  for (int e = 0; e < n_eps; ++e)
    if (!(eps[e] >= 0.0 && eps[e] <= 1.0)) return CS_ERR_INVALID_ARG;
  cs_batch_plan_t* p = new (std::nothrow) cs_batch_plan_t();
  if (!p) return CS_ERR_HIP;
  cs_status s = build_plan(count, n, counter, n_eps, eps, read_tile256_min_n(tune_cache), p);
  if (s != CS_OK) {
    if (p->dev) (void)hipFree(p->dev);
    delete p;
    return s;
  }
  *plan = p;
  return CS_OK;
}

size_t cs_batch_workspace_bytes(cs_batch_plan_handle plan) { return plan ? plan->ws_bytes : 0; }

int64_t cs_batch_hist_len(cs_batch_plan_handle plan) { return plan ? plan->hist_len : -1; }

int64_t cs_batch_hist_offset(cs_batch_plan_handle plan, int64_t k) {
  if (!plan || k < 0 || k >= plan->count) return -1;
  return plan->inst[k].hist_off;
}

cs_status cs_batch_run(cs_batch_plan_handle plan, const uint64_t* seeds, uint64_t* hist,
                       double* actions, void* workspace, size_t workspace_bytes, void* stream) {
  if (!plan || !seeds || !hist || !workspace || (plan->n_eps > 0 && !actions))
    return CS_ERR_INVALID_ARG;
  if (workspace_bytes < plan->ws_bytes) return CS_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  unsigned int* ctr = (unsigned int*)ws;
  double* coords = (double*)(ws + plan->off_coords);
  uint64_t* bits = (uint64_t*)(ws + plan->off_bits);
  cs_status s;
  if ((s = launch_fill_u64((uint64_t*)ctr, 2, 0, st)) != CS_OK) return s;
  if ((s = launch_fill_u64(hist, plan->hist_len, 0, st)) != CS_OK) return s;
  if ((s = launch_sprinkle_batch(seeds, plan->d_inst, plan->count, coords, st)) != CS_OK) return s;
  if ((s = launch_build_batch(coords, plan->d_inst, plan->d_build, plan->n_build, bits, st)) != CS_OK)
    return s;
  if ((s = run_counts(plan, bits, hist, ctr, st)) != CS_OK) return s;
  return launch_action_batch(hist, plan->d_inst, plan->count, 2, plan->d_eps, plan->n_eps, actions,
                             st);
}

cs_status cs_batch_free(cs_batch_plan_handle plan) {
  if (!plan) return CS_OK;
  hipError_t e = plan->dev ? hipFree(plan->dev) : hipSuccess;
  delete plan;
  return e == hipSuccess ? CS_OK : CS_ERR_HIP;
}

cs_status cs_batch_graph_create(cs_batch_plan_handle plan, const uint64_t* seeds, uint64_t* hist,
                                double* actions, void* workspace, size_t workspace_bytes,
                                void** graph_exec) {
  if (!graph_exec) return CS_ERR_INVALID_ARG;
  *graph_exec = nullptr;
  hipStream_t cap;
  CS_HIP_CHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  cs_status s = CS_OK;
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipStreamDestroy(cap);
    return CS_ERR_HIP;
  }
  s = cs_batch_run(plan, seeds, hist, actions, workspace, workspace_bytes, cap);
  hipError_t e = hipStreamEndCapture(cap, &g);
  (void)hipStreamDestroy(cap);
  if (s != CS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return CS_ERR_HIP;
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return CS_ERR_HIP;
  *graph_exec = (void*)ex;
  return CS_OK;
}

cs_status cs_batch_graph_launch(void* graph_exec, void* stream) {
  if (!graph_exec) return CS_ERR_INVALID_ARG;
  CS_HIP_CHECK(hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream));
  return CS_OK;
}

cs_status cs_batch_graph_destroy(void* graph_exec) {
  if (!graph_exec) return CS_OK;
  CS_HIP_CHECK(hipGraphExecDestroy((hipGraphExec_t)graph_exec));
  return CS_OK;
}

// Measures, for ensembles of `reps` 1+1 diamonds of each size in a fixed ladder, the
// MFMA counter with 128 and with 256 tiles (best of three launches each, HIP events)
// and writes the smallest size from which 256 tiles win at every larger size.
cs_status cs_autotune(const char* cache_path, void* stream) {
  if (!cache_path) return CS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int64_t ladder[] = {512, 1024, 1536, 2048, 3072, 4096, 6144, 8192};
  const int nl = (int)(sizeof(ladder) / sizeof(ladder[0]));
  const int64_t reps = 16;
  double t128[8], t256[8];
  hipEvent_t e0, e1;
  CS_HIP_CHECK(hipEventCreate(&e0));
  CS_HIP_CHECK(hipEventCreate(&e1));
  cs_status status = CS_OK;
  for (int l = 0; l < nl && status == CS_OK; ++l) {
    std::vector<int64_t> sizes(reps, ladder[l]);
    double best[2] = {1e30, 1e30};
    for (int variant = 0; variant < 2 && status == CS_OK; ++variant) {
      // variant 0: every instance on 128 tiles; variant 1: every instance on 256 tiles
      cs_batch_plan_t q;
      status = build_plan(reps, sizes.data(), CS_COUNT_MFMA, 0, nullptr,
                          variant == 0 ? (int64_t)1 << 40 : 0, &q);
      if (status != CS_OK) {
        if (q.dev) (void)hipFree(q.dev);
        break;
      }
      void* ws = nullptr;
      uint64_t* hist = nullptr;
      uint64_t* seeds = nullptr;
      if (hipMalloc(&ws, q.ws_bytes) != hipSuccess ||
          hipMalloc((void**)&hist, sizeof(uint64_t) * q.hist_len) != hipSuccess ||
          hipMalloc((void**)&seeds, sizeof(uint64_t) * reps) != hipSuccess) {
        status = CS_ERR_HIP;
      } else {
        std::vector<uint64_t> hs(reps);
        for (int64_t k = 0; k < reps; ++k) hs[k] = 0x5EEDull + 7919ull * k + 104729ull * l;
        (void)hipMemcpy(seeds, hs.data(), sizeof(uint64_t) * reps, hipMemcpyHostToDevice);
        status = cs_batch_run(&q, seeds, hist, nullptr, ws, q.ws_bytes, st);
        for (int it = 0; it < 3 && status == CS_OK; ++it) {
          unsigned int* ctr = (unsigned int*)ws;
          (void)launch_fill_u64((uint64_t*)ctr, 2, 0, st);
          (void)launch_fill_u64(hist, q.hist_len, 0, st);
          (void)hipEventRecord(e0, st);
          status = run_counts(&q, (uint64_t*)((char*)ws + q.off_bits), hist, ctr, st);
          (void)hipEventRecord(e1, st);
          if (hipEventSynchronize(e1) != hipSuccess) status = CS_ERR_HIP;
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          best[variant] = std::min(best[variant], (double)ms);
        }
      }
      if (ws) (void)hipFree(ws);
      if (hist) (void)hipFree(hist);
      if (seeds) (void)hipFree(seeds);
      if (q.dev) (void)hipFree(q.dev);
      q.dev = nullptr;
    }
    t128[l] = best[0];
    t256[l] = best[1];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status != CS_OK) return status;
  int64_t thr = (int64_t)1 << 40;
  for (int l = nl - 1; l >= 0; --l) {
    if (t256[l] < t128[l]) thr = ladder[l];
    else break;
  }
  FILE* f = fopen(cache_path, "w");
  if (!f) return CS_ERR_INVALID_ARG;
  fprintf(f, "{\n  \"tile256_min_n\": %lld,\n  \"instances_per_size\": %lld,\n  \"ms\": [",
          (long long)(thr > kBatchMaxN ? kBatchMaxN + 1 : thr), (long long)reps);
  for (int l = 0; l < nl; ++l)
    fprintf(f, "%s\n    {\"n\": %lld, \"tile128\": %.4f, \"tile256\": %.4f}", l ? "," : "",
            (long long)ladder[l], t128[l], t256[l]);
  fprintf(f, "\n  ]\n}\n");
  fclose(f);
  return CS_OK;
}

}  // extern "C"
