// Ensembles of independent 1+1 diamonds: plan, run, HIP-graph capture and the tile
// autotuner.  (The thesis averages its action measurements over ensembles of
// causal sets; here the ensemble is one pipeline of four launches.)
//
// Plan: per-instance offsets into three concatenated buffers (coordinates, matrices,
// histograms), the builder's work lists (items of 4x2 blocks of 64x64, per XCD) and
// the counters' work lists (one item per row panel I of output tiles, i.e. all tiles
// (I, J >= I) of an instance, so a workgroup keeps one instance's histogram in LDS for
// a whole panel), dealt to one queue per XCD: whole instances, largest first to the
// least loaded queue, so the queues balance instances of very different sizes while the
// workgroups of one XCD work through one instance at a time and share its panels in that
// XCD's L2 (a workgroup that runs out of its own queue takes from the others).  Against
// one queue of row panels sorted by cost across all instances, this fetches 2.5x fewer
// bytes from HBM per launch.  These tables live in device memory owned
// by the plan, uploaded once at plan time, so a run only enqueues kernels: fill,
// sprinkle, build, count (one persistent launch per tile configuration in use), action.
//
// Tile configuration per instance: the counter's configuration for the instance's size
// bucket.  The candidates are, for the MFMA counters, 128x128 tiles with one or two
// workgroups per CU and 256x256 tiles (one per CU); for the bitset counter, the dense
// product on every tile or the related-pair tiles with two thresholds, two workgroups
// per CU, and the related-pair tiles with one.  cs_autotune times every candidate on
// the device per (counter, bucket) and stores the fastest in a JSON cache, one entry per
// line; cs_batch_plan reads its counter's entries from that file when given its path
// and falls back to fixed defaults for the rest.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "common.h"

using namespace cs;

namespace {

constexpr int kMaxSlots = 8;  // distinct tile configurations in one plan

// Size buckets of the tuner: [lo, hi] and the centre of the sizes timed for each.
constexpr int kBuckets = 4;
constexpr int64_t kBucketLo[kBuckets] = {2, 1024, 2048, 4096};
constexpr int64_t kBucketHi[kBuckets] = {1023, 2047, 4095, kBatchMaxN};
constexpr int64_t kBucketProbe[kBuckets] = {768, 1536, 3072, 6144};

int bucket_of(int64_t n) {
  for (int b = 0; b < kBuckets; ++b)
    if (n <= kBucketHi[b]) return b;
  return kBuckets - 1;
}

// Counter slots of the cache: 0 bitset, 1 int8 MFMA, 2 fp4 MFMA.
constexpr const char* kCounterName[3] = {"bitset", "mfma", "mfma_fp4"};

bool same_tile(const BatchTile& a, const BatchTile& b) {
  return a.mode == b.mode && a.per_cu == b.per_cu && a.pair_max == b.pair_max;
}

// Candidates the tuner times per counter family.
const BatchTile kMfmaCandidates[] = {{2, 2, 0}, {2, 1, 0}, {4, 1, 0}};
const BatchTile kBitsetCandidates[] = {{0, 2, -1}, {0, 2, 1152}, {0, 2, 2304}, {0, 1, 2304}};

// Defaults without a cache entry: MFMA 128 tiles, two per CU, below 4096 points and 256
// tiles from there; the bitset counter on related-pair tiles with the largest task list.
BatchTile default_tile(int counter, int64_t n) {
  if (counter == CS_COUNT_BITSET) return {0, 2, 2304};
  (void)n;  // 128-row tiles, two workgroups per CU: the tuner's choice at every size
  return BatchTile{2, 2, 0};
}

struct TuneTable {
  bool have[3][kBuckets] = {};
  BatchTile cfg[3][kBuckets] = {};
  double ms[3][kBuckets] = {};
  int64_t reps[3][kBuckets] = {};  // instances of the probe ensemble
};

int counter_slot(int counter) {
  return counter == CS_COUNT_BITSET ? 0 : (counter == CS_COUNT_MFMA ? 1 : 2);
}

long long field_ll(const char* entry, const char* end, const char* key, bool* ok) {
  const char* k = strstr(entry, key);
  if (!k || k > end) {
    *ok = false;
    return 0;
  }
  const char* colon = strchr(k, ':');
  if (!colon || colon > end) {
    *ok = false;
    return 0;
  }
  return atoll(colon + 1);
}

// Reads the entries {"counter": ..., "n_lo": ..., "mode": ..., "per_cu": ..., "pair_max":
// ..., "ms": ...} of a cache written by cs_autotune; unknown or malformed entries are
// skipped, a missing file gives an empty table.
TuneTable read_tune(const char* path) {
  TuneTable t;
  if (!path || !*path) return t;
  FILE* f = fopen(path, "r");
  if (!f) return t;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  fclose(f);
  const char* p = text.c_str();
  while ((p = strstr(p, "{\"counter\": \"")) != nullptr) {
    const char* name = p + strlen("{\"counter\": \"");
    const char* end = strchr(name, '}');
    if (!end) break;
    int c = -1;
    for (int q = 0; q < 3; ++q) {
      const size_t L = strlen(kCounterName[q]);
      if (strncmp(name, kCounterName[q], L) == 0 && name[L] == '"') c = q;
    }
    bool ok = c >= 0;
    const long long lo = field_ll(name, end, "\"n_lo\"", &ok);
    const long long mode = field_ll(name, end, "\"mode\"", &ok);
    const long long per_cu = field_ll(name, end, "\"per_cu\"", &ok);
    const long long pmax = field_ll(name, end, "\"pair_max\"", &ok);
    const char* msk = strstr(name, "\"ms\"");
    const double ms = (msk && msk < end) ? atof(strchr(msk, ':') + 1) : 0.0;
    int b = -1;
    for (int q = 0; q < kBuckets; ++q)
      if (kBucketLo[q] == lo) b = q;
    const bool mode_ok = c == 0 ? mode == 0 : (mode == 2 || mode == 4);
    if (ok && b >= 0 && mode_ok && (per_cu == 1 || per_cu == 2) && !(mode == 4 && per_cu != 1)) {
      bool has_reps = true;
      const long long reps = field_ll(name, end, "\"probe_instances\"", &has_reps);
      t.have[c][b] = true;
      t.cfg[c][b] = {(int)mode, (int)per_cu, (int)pmax};
      t.ms[c][b] = ms;
      t.reps[c][b] = has_reps ? reps : 0;
    }
    p = end;
  }
  return t;
}

bool write_tune(const char* path, const TuneTable& t) {
  FILE* f = fopen(path, "w");
  if (!f) return false;
  fprintf(f, "{\n  \"format\": \"causal-batch-tune-2\",\n  \"entries\": [");
  bool first = true;
  for (int c = 0; c < 3; ++c)
    for (int b = 0; b < kBuckets; ++b) {
      if (!t.have[c][b]) continue;
      const BatchTile& x = t.cfg[c][b];
      fprintf(f, "%s\n    {\"counter\": \"%s\", \"n_lo\": %lld, \"n_hi\": %lld, \"mode\": %d, "
                 "\"tile\": %d, \"per_cu\": %d, \"pair_max\": %d, \"ms\": %.5f, "
                 "\"probe_n\": %lld, \"probe_instances\": %lld}",
              first ? "" : ",", kCounterName[c], (long long)kBucketLo[b],
              (long long)kBucketHi[b], x.mode, x.mode == 4 ? 256 : 128, x.per_cu, x.pair_max,
              t.ms[c][b], (long long)kBucketProbe[b], (long long)t.reps[c][b]);
      first = false;
    }
  fprintf(f, "\n  ]\n}\n");
  return fclose(f) == 0;
}

}  // namespace

struct cs_batch_plan_t {
  int64_t count = 0;
  int counter = CS_COUNT_MFMA;
  int n_eps = 0;
  std::vector<BatchInst> inst;
  int64_t coords_len = 0, bits_len = 0, hist_len = 0;
  int64_t n_build = 0;
  int nslots = 0;
  BatchTile slot_cfg[kMaxSlots] = {};
  int64_t n_items[kMaxSlots] = {};
  BatchQueues queues[kMaxSlots] = {};
  size_t ws_bytes = 0, off_coords = 0, off_bits = 0;
  void* dev = nullptr;              // device tables
  BatchInst* d_inst = nullptr;
  double* d_eps = nullptr;
  uint32_t* d_build = nullptr;
  uint32_t* d_items[kMaxSlots] = {};
  int device = 0;
};

namespace {

size_t take(size_t* off, size_t bytes) {
  size_t o = *off;
  *off = align_up(*off + bytes, 256);
  return o;
}

// tune: the cache's choices (entries it lacks use default_tile); force: if not null,
// every instance takes this configuration (the tuner's candidates).
cs_status build_plan(int64_t count, const int64_t* n, int counter, int n_eps, const double* eps,
                     const TuneTable& tune, const BatchTile* force, cs_batch_plan_t* p) {
  p->count = count;
  p->counter = counter;
  p->n_eps = n_eps;
  p->inst.resize(count);
  std::vector<std::vector<uint32_t>> bitems(count);  // builder items of each instance
  struct Item {
    uint32_t packed;
    int64_t cost;
  };
  std::vector<Item> items[kMaxSlots];
  const int cslot = counter_slot(counter);
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
    // Builder items (row group g: row blocks kBuildRowBlocks g + r; column blocks bj0 + c)
    // in patches of kBuildPatch x kBuildPatch blocks: a patch writes whole 128-byte lines
    // of its rows' words and of its transposed words, so the lines are complete while the
    // XCD that builds the instance holds them in its L2.
    static_assert(kBuildPatch % kBuildRowBlocks == 0 && kBuildPatch % kBuildColBlocks == 0 &&
                      kBuildRowBlocks % kBuildColBlocks == 0, "builder items tile the patches");
    constexpr int64_t G = kBuildPatch / kBuildRowBlocks;  // row groups per patch
    for (int64_t pr = 0; pr * kBuildPatch < nb; ++pr)
      for (int64_t pc = pr; pc * kBuildPatch < nb; ++pc)
        for (int64_t g = pr * G; g < pr * G + G && g * kBuildRowBlocks < nb; ++g)
          for (int64_t bj = std::max(pc * kBuildPatch, g * kBuildRowBlocks);
               bj < std::min((pc + 1) * kBuildPatch, nb); bj += kBuildColBlocks)
            bitems[k].push_back((uint32_t)(k << 16 | g << 8 | bj));
    const int b = bucket_of(d.n);
    const BatchTile cfg = force ? *force
                          : (tune.have[cslot][b] ? tune.cfg[cslot][b] : default_tile(counter, d.n));
    int slot = -1;
    for (int q = 0; q < p->nslots; ++q)
      if (same_tile(p->slot_cfg[q], cfg)) slot = q;
    if (slot < 0) {
      if (p->nslots == kMaxSlots) return CS_ERR_UNSUPPORTED;
      slot = p->nslots++;
      p->slot_cfg[slot] = cfg;
    }
    const int64_t BM = cfg.mode == 4 ? 256 : 128;
    const int64_t T = ceil_div(d.n, BM);
    for (int64_t I = 0; I < T; ++I)  // row panel I: tiles (I, J) for J = I .. T-1
      items[slot].push_back({(uint32_t)(k << 16 | I << 8), (T - I) * (T - I + 1) / 2 * BM * BM * BM});
  }
  p->coords_len = coff;
  p->bits_len = boff;
  p->hist_len = hoff;
  // Builder lists, one per XCD: whole instances dealt largest first to the shortest list,
  // so that every line of a matrix is written from one L2 (partial lines written back
  // from several XCDs multiplied the builder's HBM writes).  Workgroup b takes list
  // b mod 8 (the XCD that the dispatcher gives it), entries kBuildWaves (b div 8) + wave;
  // lists are padded with kNoBuildItem to one length, a multiple of kBuildWaves.
  std::vector<uint32_t> build;
  {
    std::vector<int64_t> order(count);
    for (int64_t k = 0; k < count; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
      return bitems[a].size() > bitems[b].size();
    });
    std::vector<uint32_t> lists[kBatchQueues];
    for (int64_t k : order) {
      int best = 0;
      for (int x = 1; x < kBatchQueues; ++x)
        if (lists[x].size() < lists[best].size()) best = x;
      lists[best].insert(lists[best].end(), bitems[k].begin(), bitems[k].end());
    }
    size_t len = 0;
    for (auto& l : lists) len = std::max(len, l.size());
    len = (len + kBuildWaves - 1) / kBuildWaves * kBuildWaves;
    build.assign(len * kBatchQueues, kNoBuildItem);
    for (int x = 0; x < kBatchQueues; ++x)
      std::copy(lists[x].begin(), lists[x].end(), build.begin() + x * len);
  }
  p->n_build = (int64_t)build.size();
  for (int s = 0; s < p->nslots; ++s) {
    // One queue per XCD holding whole instances, dealt largest first to the least loaded
    // queue; a queue runs its instances one after another (largest first), each
    // instance's row panels longest first, so the workgroups of one XCD work on the same
    // matrix at the same time and share its panels through that XCD's L2.
    std::vector<int64_t> work(count, 0);
    std::vector<std::vector<Item>> per(count);
    for (const Item& it : items[s]) {
      work[it.packed >> 16] += it.cost;
      per[it.packed >> 16].push_back(it);
    }
    std::vector<int64_t> order;
    for (int64_t k = 0; k < count; ++k)
      if (!per[k].empty()) order.push_back(k);
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return work[a] > work[b]; });
    std::vector<int> queue_of(count, 0);
    int64_t load[kBatchQueues] = {};
    for (int64_t k : order) {
      int best = 0;
      for (int x = 1; x < kBatchQueues; ++x)
        if (load[x] < load[best]) best = x;
      queue_of[k] = best;
      load[best] += work[k];
    }
    std::vector<Item> sorted;
    sorted.reserve(items[s].size());
    for (int x = 0; x < kBatchQueues; ++x) {
      p->queues[s].off[x] = (uint32_t)sorted.size();
      for (int64_t k : order)
        if (queue_of[k] == x) {
          std::stable_sort(per[k].begin(), per[k].end(),
                           [](const Item& a, const Item& b) { return a.cost > b.cost; });
          sorted.insert(sorted.end(), per[k].begin(), per[k].end());
        }
    }
    p->queues[s].off[kBatchQueues] = (uint32_t)sorted.size();
    items[s].swap(sorted);
    p->n_items[s] = (int64_t)items[s].size();
  }

  // Caller workspace: [tile counters, one per slot][coordinates][matrices].
  size_t off = 0;
  static_assert(sizeof(unsigned int) * kMaxSlots * kBatchQueues == 256, "work counters");
  take(&off, 256);
  p->off_coords = take(&off, sizeof(double) * (size_t)coff);
  p->off_bits = take(&off, sizeof(uint64_t) * (size_t)boff);
  p->ws_bytes = off;

  // Device tables owned by the plan.
  size_t doff = 0;
  size_t o_inst = take(&doff, sizeof(BatchInst) * count);
  size_t o_eps = take(&doff, sizeof(double) * (n_eps > 0 ? n_eps : 1));
  size_t o_build = take(&doff, sizeof(uint32_t) * build.size());
  size_t o_items[kMaxSlots];
  for (int s = 0; s < p->nslots; ++s) o_items[s] = take(&doff, sizeof(uint32_t) * items[s].size());
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
  for (int s = 0; s < p->nslots; ++s) {
    p->d_items[s] = (uint32_t*)(b + o_items[s]);
    uint32_t* dst = (uint32_t*)(host.data() + o_items[s]);
    for (size_t q = 0; q < items[s].size(); ++q) dst[q] = items[s][q].packed;
  }
  CS_HIP_CHECK(hipMemcpy(p->dev, host.data(), doff, hipMemcpyHostToDevice));
  return CS_OK;
}

cs_status run_counts(cs_batch_plan_t* p, const uint64_t* bits, uint64_t* hist, unsigned int* ctr,
                     hipStream_t st) {
  for (int s = 0; s < p->nslots; ++s) {
    if (!p->n_items[s]) continue;
    cs_status r = launch_count_batch(p->slot_cfg[s], p->counter == CS_COUNT_MFMA_FP4, bits,
                                     p->d_inst, p->d_items[s], p->queues[s], hist,
                                     ctr + s * kBatchQueues, st);
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
  cs_status s = build_plan(count, n, counter, n_eps, eps, read_tune(tune_cache), nullptr, p);
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

int64_t cs_batch_coords_offset(cs_batch_plan_handle plan, int64_t k) {
  if (!plan || k < 0 || k >= plan->count) return -1;
  return (int64_t)plan->off_coords + (int64_t)sizeof(double) * plan->inst[k].coord_off;
}

int64_t cs_batch_bits_offset(cs_batch_plan_handle plan, int64_t k) {
  if (!plan || k < 0 || k >= plan->count) return -1;
  return (int64_t)plan->off_bits + (int64_t)sizeof(uint64_t) * plan->inst[k].bits_off;
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
  // the sprinkle kernel also clears the histograms and the work counters
  if ((s = launch_sprinkle_batch(seeds, plan->d_inst, plan->count, coords, hist, (uint64_t*)ctr,
                                 kMaxSlots * kBatchQueues / 2, st)) != CS_OK)
    return s;
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

// For each requested (counter, bucket): an ensemble of `reps` diamonds of the bucket's
// probe size, every tile configuration of the counter's candidates forced on all of them,
// the counting launches timed (best of three, HIP events); the fastest is stored.
cs_status cs_autotune(const char* cache_path, int64_t n_bucket, int counter, void* stream) {
  if (!cache_path) return CS_ERR_INVALID_ARG;
  if (counter != -1 && counter != CS_COUNT_BITSET && counter != CS_COUNT_MFMA &&
      counter != CS_COUNT_MFMA_FP4)
    return CS_ERR_UNSUPPORTED;
  if (n_bucket != 0 && (n_bucket < 2 || n_bucket > kBatchMaxN)) return CS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  TuneTable table = read_tune(cache_path);
  const int cus = device_cu_count();
  hipEvent_t e0, e1;
  CS_HIP_CHECK(hipEventCreate(&e0));
  CS_HIP_CHECK(hipEventCreate(&e1));
  cs_status status = CS_OK;
  const int counters[3] = {CS_COUNT_BITSET, CS_COUNT_MFMA, CS_COUNT_MFMA_FP4};
  for (int ci = 0; ci < 3 && status == CS_OK; ++ci) {
    const int c = counters[ci];
    if (counter != -1 && counter != c) continue;
    const BatchTile* cand = c == CS_COUNT_BITSET ? kBitsetCandidates : kMfmaCandidates;
    const int ncand = c == CS_COUNT_BITSET
                          ? (int)(sizeof(kBitsetCandidates) / sizeof(kBitsetCandidates[0]))
                          : (int)(sizeof(kMfmaCandidates) / sizeof(kMfmaCandidates[0]));
    for (int b = 0; b < kBuckets && status == CS_OK; ++b) {
      if (n_bucket != 0 && bucket_of(n_bucket) != b) continue;
      // Enough instances that the row-panel items of 128-row tiles fill every CU sixteen
      // times over, as in a full ensemble (a handful of instances would leave most CUs
      // idle and favour the wrong occupancy; eight times over left candidates within the
      // timing noise of each other that differ by 8 % in a full ensemble).
      const int64_t reps = std::max<int64_t>(16, ceil_div(16 * (int64_t)cus,
                                                          ceil_div(kBucketProbe[b], 128)));
      // Sizes spread evenly over the bucket, centred on its probe size, as in an ensemble
      // of uneven instances (identical ones would all end at once and favour other tiles).
      const int64_t plo = 2 * kBucketProbe[b] - kBucketHi[b], phi = kBucketHi[b];
      std::vector<int64_t> sizes(reps);
      for (int64_t k = 0; k < reps; ++k) sizes[k] = plo + (phi - plo) * k / (reps - 1);
      double best_ms = 1e30;
      int best = -1;
      for (int v = 0; v < ncand && status == CS_OK; ++v) {
        cs_batch_plan_t q;
        status = build_plan(reps, sizes.data(), c, 0, nullptr, TuneTable{}, &cand[v], &q);
        void* ws = nullptr;
        uint64_t* hist = nullptr;
        uint64_t* seeds = nullptr;
        double ms_v = 1e30;
        if (status == CS_OK &&
            (hipMalloc(&ws, q.ws_bytes) != hipSuccess ||
             hipMalloc((void**)&hist, sizeof(uint64_t) * q.hist_len) != hipSuccess ||
             hipMalloc((void**)&seeds, sizeof(uint64_t) * reps) != hipSuccess))
          status = CS_ERR_HIP;
        if (status == CS_OK) {
          std::vector<uint64_t> hs(reps);
          for (int64_t k = 0; k < reps; ++k) hs[k] = 0x5EEDull + 7919ull * k + 104729ull * b;
          if (hipMemcpy(seeds, hs.data(), sizeof(uint64_t) * reps, hipMemcpyHostToDevice) !=
              hipSuccess)
            status = CS_ERR_HIP;
          if (status == CS_OK) status = cs_batch_run(&q, seeds, hist, nullptr, ws, q.ws_bytes, st);
          for (int it = 0; it < 5 && status == CS_OK; ++it) {
            unsigned int* ctr = (unsigned int*)ws;
            status = launch_fill_u64((uint64_t*)ctr, kMaxSlots * kBatchQueues / 2, 0, st);
            if (status == CS_OK) status = launch_fill_u64(hist, q.hist_len, 0, st);
            if (status != CS_OK) break;
            (void)hipEventRecord(e0, st);
            status = run_counts(&q, (uint64_t*)((char*)ws + q.off_bits), hist, ctr, st);
            (void)hipEventRecord(e1, st);
            if (hipEventSynchronize(e1) != hipSuccess) status = CS_ERR_HIP;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            ms_v = std::min(ms_v, (double)ms);
          }
        }
        if (ws) (void)hipFree(ws);
        if (hist) (void)hipFree(hist);
        if (seeds) (void)hipFree(seeds);
        if (q.dev) (void)hipFree(q.dev);
        q.dev = nullptr;
        if (status == CS_OK && ms_v < best_ms) {
          best_ms = ms_v;
          best = v;
        }
      }
      if (status == CS_OK && best >= 0) {
        const int cs_ = counter_slot(c);
        table.have[cs_][b] = true;
        table.cfg[cs_][b] = cand[best];
        table.ms[cs_][b] = best_ms;
        table.reps[cs_][b] = reps;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status != CS_OK) return status;
  return write_tune(cache_path, table) ? CS_OK : CS_ERR_INVALID_ARG;
}

}  // extern "C"
