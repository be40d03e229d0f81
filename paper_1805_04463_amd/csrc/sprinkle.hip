// Sprinkling and time ordering on the GPU (App. A "Causal Set Sprinklings";
// Sec. 3.2 "Pairwise Relations": label elements so that no later index precedes
// an earlier one).
//
// Pipeline per call: generate raw SoA coordinates + a 64-bit time key per point
// -> bitonic sort of (key, generation index) pairs (LDS chunks of 2048 + global
// merge steps) -> gather the coordinate planes into sorted order.  Sets of at most
// 8192 points skip the sort and the gather: each point's rank is counted over all
// keys and its planes are written there.
// The 3+1 diamond is sampled by rejection: candidates are flagged, counted per
// block, scanned, and the first n accepted are scattered in candidate order.
#include "common.h"

namespace cs {
namespace {

constexpr int kBlock = 256;
constexpr int kSortChunk = 2048;  // elements sorted per LDS pass (1024 threads)

// Candidate budget of the rejection samplers of the diamonds of height 1: the
// acceptance probability is the diamond's volume in the unit box, pi/24 (3+1) or
// pi/12 (2+1); the budget covers the mean plus 12 standard deviations, and a
// one-workgroup tail kernel handles any shortfall.
bool is_rejection(int region) { return region == CS_MINK4_DIAMOND || region == CS_MINK3_DIAMOND; }

int64_t mink_candidates(int region, int64_t n) {
  const double p = region == CS_MINK3_DIAMOND ? 0.26179938779914941   // pi / 12
                                              : 0.13089969389957471;  // pi / 24
  double m = (double)n / p + 12.0 * sqrt((double)n * (1.0 - p)) / p + 4096.0;
  return align_up((size_t)m, kBlock);
}

int64_t pow2_at_least(int64_t n) {
  int64_t p = 2;
  while (p < n) p <<= 1;
  return p;
}

struct SprinkleWs {
  double* raw;
  uint64_t* keys;
  uint32_t* gens;
  uint32_t* blk_count;   // rejection samplers only
  uint64_t* blk_offset;  // rejection samplers only (exclusive scan), plus [nblk] = total
};

size_t layout(int region, int64_t n, void* base, SprinkleWs* w) {
  const int planes = coord_planes(region);
  const int64_t P = pow2_at_least(n);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  size_t o_raw = take(sizeof(double) * planes * n);
  size_t o_keys = take(sizeof(uint64_t) * P);
  size_t o_gens = take(sizeof(uint32_t) * P);
  size_t o_cnt = 0, o_off = 0;
  if (is_rejection(region)) {
    int64_t nblk = mink_candidates(region, n) / kBlock;
    o_cnt = take(sizeof(uint32_t) * nblk);
    o_off = take(sizeof(uint64_t) * (nblk + 1));
  }
  if (w) {
    char* b = (char*)base;
    w->raw = (double*)(b + o_raw);
    w->keys = (uint64_t*)(b + o_keys);
    w->gens = (uint32_t*)(b + o_gens);
    w->blk_count = is_rejection(region) ? (uint32_t*)(b + o_cnt) : nullptr;
    w->blk_offset = is_rejection(region) ? (uint64_t*)(b + o_off) : nullptr;
  }
  return off;
}

// ---------------------------------------------------------------------------
// 1+1 diamond: u = U(2g), v = U(2g+1); key = exact integer (u + v) * 2^53.
// ---------------------------------------------------------------------------
__global__ void k_sprinkle_mink2(uint64_t skey, int64_t n, int64_t P, double* __restrict__ raw,
                                 uint64_t* __restrict__ keys, uint32_t* __restrict__ gens) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= P) return;
  if (g < n) {
    uint64_t ku = sm_output(skey, 2 * (uint64_t)g) >> 11;
    uint64_t kv = sm_output(skey, 2 * (uint64_t)g + 1) >> 11;
    raw[g] = (double)ku * 0x1.0p-53;
    raw[n + g] = (double)kv * 0x1.0p-53;
    keys[g] = ku + kv;
    gens[g] = (uint32_t)g;
  } else {
    keys[g] = ~0ull;
    gens[g] = 0xFFFFFFFFu;
  }
}

// ---------------------------------------------------------------------------
// D-dimensional diamond of height 1 (D = 3 or 4) by rejection from [0,1) x
// [-1/2,1/2)^(D-1): candidate c takes draws D c .. D c + D-1 of the stream.
// ---------------------------------------------------------------------------
struct Cand {
  double t, x, y, z;
  uint64_t kt;
  bool ok;
};

template <int D>
__device__ inline Cand mink_candidate(uint64_t skey, uint64_t c) {
  Cand r;
  r.kt = sm_output(skey, D * c) >> 11;
  r.t = (double)r.kt * 0x1.0p-53;
  r.x = unit53(sm_output(skey, D * c + 1)) - 0.5;
  r.y = unit53(sm_output(skey, D * c + 2)) - 0.5;
  r.z = D == 4 ? unit53(sm_output(skey, D * c + 3)) - 0.5 : 0.0;
  double one_t = 1.0 - r.t;
  double rad = r.t < one_t ? r.t : one_t;
  double rr = __dadd_rn(__dmul_rn(r.x, r.x), __dmul_rn(r.y, r.y));
  if (D == 4) rr = __dadd_rn(rr, __dmul_rn(r.z, r.z));
  r.ok = rr < __dmul_rn(rad, rad);
  return r;
}

// Block-wide exclusive rank of `flag` among the block's threads, and the block total.
__device__ inline uint32_t block_rank(bool flag, uint32_t* total, uint32_t* s_wave) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint64_t m = __ballot(flag);
  uint32_t below = __popcll(m & ((1ull << lane) - 1ull));
  if (lane == 0) s_wave[wave] = (uint32_t)__popcll(m);
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    if (w < wave) base += s_wave[w];
    tot += s_wave[w];
  }
  __syncthreads();
  *total = tot;
  return base + below;
}

template <int D>
__global__ void k_mink_count(uint64_t skey, uint32_t* __restrict__ blk_count) {
  __shared__ uint32_t s_wave[kBlock / 64];
  uint64_t c = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  Cand r = mink_candidate<D>(skey, c);
  uint32_t tot;
  block_rank(r.ok, &tot, s_wave);
  if (threadIdx.x == 0) blk_count[blockIdx.x] = tot;
}

// Exclusive scan of nblk block counts by one workgroup of 1024 threads.
__global__ void k_scan_counts(const uint32_t* __restrict__ cnt, int64_t nblk,
                              uint64_t* __restrict__ off) {
  __shared__ uint64_t s[1024];
  uint64_t carry = 0;
  for (int64_t base = 0; base < nblk; base += 1024) {
    int64_t i = base + threadIdx.x;
    uint64_t v = i < nblk ? cnt[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {  // Hillis-Steele inclusive scan
      uint64_t a = threadIdx.x >= (unsigned)d ? s[threadIdx.x - d] : 0;
      __syncthreads();
      s[threadIdx.x] += a;
      __syncthreads();
    }
    if (i < nblk) off[i] = carry + s[threadIdx.x] - v;
    carry += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) off[nblk] = carry;
}

template <int D>
__device__ inline void put(const Cand& r, uint64_t rank, int64_t n, double* raw, uint64_t* keys,
                            uint32_t* gens) {
  raw[rank] = r.t;
  raw[n + rank] = r.x;
  raw[2 * n + rank] = r.y;
  if (D == 4) raw[3 * n + rank] = r.z;
  keys[rank] = r.kt;
  gens[rank] = (uint32_t)rank;
}

template <int D>
__global__ void k_mink_scatter(uint64_t skey, int64_t n, const uint64_t* __restrict__ blk_off,
                                double* __restrict__ raw, uint64_t* __restrict__ keys,
                                uint32_t* __restrict__ gens) {
  __shared__ uint32_t s_wave[kBlock / 64];
  uint64_t c = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  Cand r = mink_candidate<D>(skey, c);
  uint32_t tot;
  uint32_t local = block_rank(r.ok, &tot, s_wave);
  uint64_t rank = blk_off[blockIdx.x] + local;
  if (r.ok && rank < (uint64_t)n) put<D>(r, rank, n, raw, keys, gens);
}

// Continues candidates after the budget if (improbably) fewer than n were accepted.
// One workgroup; bounded number of rounds.
template <int D>
__global__ void k_mink_tail(uint64_t skey, int64_t n, int64_t M, const uint64_t* __restrict__ total,
                             double* __restrict__ raw, uint64_t* __restrict__ keys,
                             uint32_t* __restrict__ gens) {
  __shared__ uint32_t s_wave[kBlock / 64];
  uint64_t have = *total;
  const int64_t kMaxRounds = 1ll << 22;
  for (int64_t round = 0; have < (uint64_t)n && round < kMaxRounds; ++round) {
    uint64_t c = (uint64_t)M + (uint64_t)round * kBlock + threadIdx.x;
    Cand r = mink_candidate<D>(skey, c);
    uint32_t tot;
    uint32_t local = block_rank(r.ok, &tot, s_wave);
    uint64_t rank = have + local;
    if (r.ok && rank < (uint64_t)n) put<D>(r, rank, n, raw, keys, gens);
    have += tot;
  }
}

__global__ void k_pad_keys(int64_t n, int64_t P, uint64_t* __restrict__ keys,
                           uint32_t* __restrict__ gens) {
  int64_t g = n + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < P) {
    keys[g] = ~0ull;
    gens[g] = 0xFFFFFFFFu;
  }
}

// ---------------------------------------------------------------------------
// 1+1 de Sitter slab: the density sec^2(eta) = d tan(eta)/d eta makes x = tan(eta)
// uniform, x = (2u - 1) tan(eta0) (one rounding); eta = atan(x); theta = 2 pi w.
// Sorted by x, which orders the points by eta.
// ---------------------------------------------------------------------------
__global__ void k_sprinkle_ds2(uint64_t skey, double X, int64_t n, int64_t P,
                               double* __restrict__ raw, uint64_t* __restrict__ keys,
                               uint32_t* __restrict__ gens) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= P) return;
  if (g >= n) {
    keys[g] = ~0ull;
    gens[g] = 0xFFFFFFFFu;
    return;
  }
  const double two_pi = 2.0 * 3.141592653589793;  // twice the double nearest pi (exact)
  double u = unit53(sm_output(skey, 2 * (uint64_t)g));
  double w = unit53(sm_output(skey, 2 * (uint64_t)g + 1));
  double x = __dmul_rn(__dsub_rn(__dmul_rn(2.0, u), 1.0), X);
  raw[g] = x;
  raw[n + g] = atan(x);
  raw[2 * n + g] = __dmul_rn(two_pi, w);
  keys[g] = order_bits(x);
  gens[g] = (uint32_t)g;
}

// ---------------------------------------------------------------------------
// 3+1 de Sitter slab: x = tan(eta) from the inverse CDF of (1 + x^2) dx,
// x = 2 sinh(asinh(3y/2)/3); direction on S^3 by cube rejection, normalised.
// ---------------------------------------------------------------------------
__global__ void k_sprinkle_ds4(uint64_t skey_t, uint64_t skey_s, double X, int64_t n, int64_t P,
                               double* __restrict__ raw, uint64_t* __restrict__ keys,
                               uint32_t* __restrict__ gens) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= P) return;
  if (g >= n) {
    keys[g] = ~0ull;
    gens[g] = 0xFFFFFFFFu;
    return;
  }
  double Y = __dadd_rn(X, __ddiv_rn(__dmul_rn(__dmul_rn(X, X), X), 3.0));
  double u = unit53(sm_output(skey_t, (uint64_t)g));
  double y = __dmul_rn(__dsub_rn(__dmul_rn(2.0, u), 1.0), Y);
  double x = __dmul_rn(2.0, sinh(__ddiv_rn(asinh(__dmul_rn(1.5, y)), 3.0)));
  double ce = __ddiv_rn(1.0, __dsqrt_rn(__dadd_rn(1.0, __dmul_rn(x, x))));
  double se = __dmul_rn(x, ce);
  uint64_t ps = sm_output(skey_s, (uint64_t)g);
  double a0 = 1.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, r2 = 1.0;
  for (int k = 0; k < kSphereTries; ++k) {
    double b0 = __dsub_rn(__dmul_rn(2.0, unit53(sm_output(ps, 4 * (uint64_t)k + 0))), 1.0);
    double b1 = __dsub_rn(__dmul_rn(2.0, unit53(sm_output(ps, 4 * (uint64_t)k + 1))), 1.0);
    double b2 = __dsub_rn(__dmul_rn(2.0, unit53(sm_output(ps, 4 * (uint64_t)k + 2))), 1.0);
    double b3 = __dsub_rn(__dmul_rn(2.0, unit53(sm_output(ps, 4 * (uint64_t)k + 3))), 1.0);
    double q = __dadd_rn(__dmul_rn(b0, b0), __dmul_rn(b1, b1));
    q = __dadd_rn(q, __dmul_rn(b2, b2));
    q = __dadd_rn(q, __dmul_rn(b3, b3));
    if (q < 1.0 && q > 0x1.0p-40) {
      a0 = b0; a1 = b1; a2 = b2; a3 = b3; r2 = q;
      break;
    }
  }
  double r = __dsqrt_rn(r2);
  raw[g] = x;
  raw[n + g] = ce;
  raw[2 * n + g] = se;
  raw[3 * n + g] = __ddiv_rn(a0, r);
  raw[4 * n + g] = __ddiv_rn(a1, r);
  raw[5 * n + g] = __ddiv_rn(a2, r);
  raw[6 * n + g] = __ddiv_rn(a3, r);
  keys[g] = order_bits(x);
  gens[g] = (uint32_t)g;
}

// ---------------------------------------------------------------------------
// Bitonic sort of (key, gen) pairs, P a power of two.
// ---------------------------------------------------------------------------
__device__ inline void cmp_swap_lds(uint64_t* sk, uint32_t* sg, int i, int l, bool asc) {
  uint64_t ka = sk[i], kb = sk[l];
  uint32_t ga = sg[i], gb = sg[l];
  bool gt = key_less(kb, gb, ka, ga);  // a > b
  if (gt == asc) {
    sk[i] = kb; sk[l] = ka;
    sg[i] = gb; sg[l] = ga;
  }
}

// Orders a bitonic compare-exchange step after the previous one.  A step of distance
// j <= 64 pairs thread t (of a wave's 64) with elements inside the 128-element block
// t / 64 (in steps of 64 threads), so each block belongs to one wave: such a step needs
// only the wave's own earlier LDS writes.  Steps of larger distance, and the first step
// after another step of larger distance or after loading, synchronise the workgroup.
__device__ inline void bitonic_step_sync(bool workgroup) {
  if (workgroup) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// kfirst == 0: full sort of each chunk (k = 2 .. CH).  Otherwise: the j < CH steps of
// merge stage k = kfirst.  One thread per pair; CH/2 threads per block.
__global__ void k_bitonic_lds(uint64_t* __restrict__ keys, uint32_t* __restrict__ gens, int CH,
                              int64_t kfirst) {
  __shared__ uint64_t sk[kSortChunk];
  __shared__ uint32_t sg[kSortChunk];
  const int64_t base = (int64_t)blockIdx.x * CH;
  const int t = threadIdx.x;
  sk[t] = keys[base + t];
  sg[t] = gens[base + t];
  sk[t + CH / 2] = keys[base + t + CH / 2];
  sg[t + CH / 2] = gens[base + t + CH / 2];
  int64_t k0 = kfirst ? kfirst : 2;
  int64_t k1 = kfirst ? kfirst : CH;
  bool wide = true;  // the previous step (or the load) crossed 128-element blocks
  for (int64_t k = k0; k <= k1; k <<= 1) {
    int jstart = (int)((k >> 1) < (CH >> 1) ? (k >> 1) : (CH >> 1));
    for (int j = jstart; j > 0; j >>= 1) {
      bitonic_step_sync(wide || j >= 128);
      wide = j >= 128;
      int i = 2 * t - (t & (j - 1));
      bool asc = ((base + i) & k) == 0;
      cmp_swap_lds(sk, sg, i, i + j, asc);
    }
  }
  __syncthreads();
  keys[base + t] = sk[t];
  gens[base + t] = sg[t];
  keys[base + t + CH / 2] = sk[t + CH / 2];
  gens[base + t + CH / 2] = sg[t + CH / 2];
}

__global__ void k_bitonic_global(uint64_t* __restrict__ keys, uint32_t* __restrict__ gens,
                                 int64_t P, int64_t k, int64_t j) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P / 2) return;
  int64_t i = 2 * t - (t & (j - 1));
  int64_t l = i + j;
  bool asc = (i & k) == 0;
  uint64_t ka = keys[i], kb = keys[l];
  uint32_t ga = gens[i], gb = gens[l];
  if (key_less(kb, gb, ka, ga) == asc) {
    keys[i] = kb; keys[l] = ka;
    gens[i] = gb; gens[l] = ga;
  }
}

__global__ void k_gather(const double* __restrict__ raw, const uint32_t* __restrict__ gens,
                         int planes, int64_t n, double* __restrict__ coords) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t g = gens[i];
  for (int p = 0; p < planes; ++p) coords[(int64_t)p * n + i] = raw[(int64_t)p * n + g];
}

// ---------------------------------------------------------------------------
// Small sets: the time order by ranks.  Element g's place is the number of elements
// before it in (key, index) order, the order the sort network produces; the place is
// counted over every key and the coordinates are written straight there, which replaces
// the sort and the gather by one launch.  Sixteen lanes share an element, each comparing
// against every sixteenth key of a chunk staged in LDS (consecutive lanes read
// consecutive words, so a wave's reads hit distinct banks); the partial counts are summed
// by lane exchanges.  Each comparison is the order itself, key first and index on equal
// keys, so equal keys need no separate pass.
// ---------------------------------------------------------------------------
constexpr int kRankThreads = 256;
constexpr int kRankSplit = 16;                       // lanes per element
constexpr int kRankPer = kRankThreads / kRankSplit;  // elements per workgroup
constexpr int kRankChunk = 2048;                     // keys staged per pass
constexpr int64_t kRankMaxN = 8192;                  // n^2 comparisons: small sets only

__device__ inline uint32_t rank_lane_sum(uint32_t v) {
#pragma unroll
  for (int off = kRankSplit / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__global__ __launch_bounds__(kRankThreads) void k_rank_place(const uint64_t* __restrict__ keys,
                                                             const double* __restrict__ raw,
                                                             int planes, int64_t n,
                                                             double* __restrict__ coords) {
  __shared__ uint64_t sk[kRankChunk];
  const int s = threadIdx.x & (kRankSplit - 1);
  const int64_t g = (int64_t)blockIdx.x * kRankPer + threadIdx.x / kRankSplit;
  const bool live = g < n;
  const uint64_t kg = live ? keys[g] : 0ull;
  uint32_t before = 0;  // elements h with (key_h, h) < (key_g, g)
  for (int64_t base = 0; base < n; base += kRankChunk) {
    const int m = (int)(n - base < kRankChunk ? n - base : kRankChunk);
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += kRankThreads) sk[i] = keys[base + i];
    __syncthreads();
    const int gi = (int)(g - base);  // g's index within the chunk (any value if outside)
#pragma unroll 8
    for (int i = s; i < m; i += kRankSplit) {
      const uint64_t kh = sk[i];
      before += (kh < kg || (kh == kg && i < gi)) ? 1u : 0u;
    }
  }
  const uint32_t lt = rank_lane_sum(before);
  if (live)
    for (int p = s; p < planes; p += kRankSplit) coords[(int64_t)p * n + lt] = raw[(int64_t)p * n + g];
}

// The 1+1 diamond's time key of draw g (see k_sprinkle_mink2).
__device__ inline uint64_t mink2_key(uint64_t skey, uint64_t g) {
  return (sm_output(skey, 2 * g) >> 11) + (sm_output(skey, 2 * g + 1) >> 11);
}

// 1+1 diamonds up to kRankMaxN points: k_rank_place with the keys and coordinates taken
// straight from the counter-based generator, so the draws, the ranks and the placement
// are one launch.
__global__ __launch_bounds__(kRankThreads) void k_rank_place_mink2(uint64_t skey, int64_t n,
                                                                   double* __restrict__ coords) {
  __shared__ uint64_t sk[kRankChunk];
  const int s = threadIdx.x & (kRankSplit - 1);
  const int64_t g = (int64_t)blockIdx.x * kRankPer + threadIdx.x / kRankSplit;
  const bool live = g < n;
  const uint64_t ku = live ? sm_output(skey, 2 * (uint64_t)g) >> 11 : 0ull;
  const uint64_t kv = live ? sm_output(skey, 2 * (uint64_t)g + 1) >> 11 : 0ull;
  const uint64_t kg = ku + kv;
  uint32_t before = 0;  // elements h with (key_h, h) < (key_g, g)
  for (int64_t base = 0; base < n; base += kRankChunk) {
    const int m = (int)(n - base < kRankChunk ? n - base : kRankChunk);
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += kRankThreads) sk[i] = mink2_key(skey, (uint64_t)(base + i));
    __syncthreads();
    const int gi = (int)(g - base);  // g's index within the chunk (any value if outside)
#pragma unroll 8
    for (int i = s; i < m; i += kRankSplit) {
      const uint64_t kh = sk[i];
      before += (kh < kg || (kh == kg && i < gi)) ? 1u : 0u;
    }
  }
  const uint32_t lt = rank_lane_sum(before);
  if (live && s < 2) coords[(int64_t)s * n + lt] = (double)(s == 0 ? ku : kv) * 0x1.0p-53;
}

cs_status bitonic_sort(uint64_t* keys, uint32_t* gens, int64_t P, hipStream_t st) {
  const int CH = (int)(P < kSortChunk ? P : kSortChunk);
  const unsigned nchunks = (unsigned)(P / CH);
  hipLaunchKernelGGL(k_bitonic_lds, dim3(nchunks), dim3(CH / 2), 0, st, keys, gens, CH,
                     (int64_t)0);
  CS_LAUNCH_CHECK();
  for (int64_t k = 2 * (int64_t)CH; k <= P; k <<= 1) {
    for (int64_t j = k >> 1; j >= CH; j >>= 1) {
      unsigned blocks = (unsigned)ceil_div(P / 2, 256);
      hipLaunchKernelGGL(k_bitonic_global, dim3(blocks), dim3(256), 0, st, keys, gens, P, k, j);
      CS_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_bitonic_lds, dim3(nchunks), dim3(CH / 2), 0, st, keys, gens, CH, k);
    CS_LAUNCH_CHECK();
  }
  return CS_OK;
}

// ---------------------------------------------------------------------------
// Ensemble of 1+1 diamonds: one workgroup per instance (n <= 8192).  The time order is
// (key, generation index) with the 54-bit key of the single-instance path.  The LDS sort
// runs on one 64-bit word per point, the key's top 32 bits above the index, so each
// compare-exchange moves 16 bytes instead of 24; points whose top key bits tie (about
// one instance in thirty has such a pair) form runs that a second pass puts in
// (key, index) order, with the keys regenerated from the indices (the generator is
// counter-based).  The sorted coordinates are then regenerated the same way, so no raw
// copy is kept.
// ---------------------------------------------------------------------------
constexpr int kBatchSortThreads = 1024;
constexpr int kBatchKeyShift = 22;  // 54-bit keys: the top 32 bits go into the sort word

__global__ __launch_bounds__(kBatchSortThreads) void k_sprinkle_mink2_batch(
    const uint64_t* __restrict__ seeds, const BatchInst* __restrict__ inst,
    double* __restrict__ coords, uint64_t* __restrict__ hist, uint64_t* __restrict__ zero,
    int nzero) {
  __shared__ uint64_t sw[kBatchMaxN];  // key >> kBatchKeyShift << 32 | generation index
  const BatchInst d = inst[blockIdx.x];
  const int n = (int)d.n;
  // The pipeline's later kernels accumulate into the instance's histogram and take work
  // from counters: both start at zero, cleared here instead of by launches of their own.
  for (int m = threadIdx.x; m < n - 1; m += kBatchSortThreads) hist[d.hist_off + m] = 0;
  if (blockIdx.x == 0)
    for (int w = threadIdx.x; w < nzero; w += kBatchSortThreads) zero[w] = 0;
  int P = 2;
  while (P < n) P <<= 1;
  const uint64_t skey = sm_stream_key(seeds[blockIdx.x], kStreamMink2);
  for (int g = threadIdx.x; g < P; g += kBatchSortThreads)
    sw[g] = g < n ? (mink2_key(skey, (uint64_t)g) >> kBatchKeyShift) << 32 | (uint32_t)g : ~0ull;
  // One compare-exchange step of distance j in merge stage k through LDS: pairs t,
  // t + 1024, ... of thread t; with j <= 64 every 128-element block is still worked by
  // one wave (block b by wave b mod 16), so the step only synchronises the wave.
  bool wide = true;  // the previous step (or the load) crossed 128-element blocks
  auto lds_step = [&](int k, int j) {
    bitonic_step_sync(wide || j >= 128);
    wide = j >= 128;
    for (int t = threadIdx.x; t < P / 2; t += kBatchSortThreads) {
      const int i = 2 * t - (t & (j - 1));
      const uint64_t x = sw[i], y = sw[i + j];
      if ((x > y) == ((i & k) == 0)) {
        sw[i] = y;
        sw[i + j] = x;
      }
    }
  };
  // The steps of distance 4, 2 and 1 of stage k (and, with k = 0, the whole of stages
  // 2, 4 and 8) on 8-element chunks held in registers: one LDS read and write of each
  // element instead of three steps.  A chunk's 8 elements share the direction bit of
  // every stage k >= 8.
  auto chunk_steps = [&](int k) {
    __syncthreads();
    for (int c = threadIdx.x; c < P / 8; c += kBatchSortThreads) {
      uint64_t v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = sw[8 * c + e];
      auto cx = [&](int e, int j, bool asc) {
        const uint64_t x = v[e], y = v[e + j];
        const bool sw_ = (x > y) == asc;
        v[e] = sw_ ? y : x;
        v[e + j] = sw_ ? x : y;
      };
      if (k == 0) {
#pragma unroll
        for (int kk = 2; kk <= 8; kk <<= 1)
#pragma unroll
          for (int j = kk >> 1; j > 0; j >>= 1)
#pragma unroll
            for (int e = 0; e < 8; ++e)
              if ((e & j) == 0) cx(e, j, ((8 * c + e) & kk) == 0);
      } else {
        const bool asc = ((8 * c) & k) == 0;
#pragma unroll
        for (int j = 4; j > 0; j >>= 1)
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if ((e & j) == 0) cx(e, j, asc);
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) sw[8 * c + e] = v[e];
    }
    wide = true;
  };
  if (P >= 8) {
    chunk_steps(0);
    for (int k = 16; k <= P; k <<= 1) {
      for (int j = k >> 1; j >= 8; j >>= 1) lds_step(k, j);
      chunk_steps(k);
    }
  } else {
    for (int k = 2; k <= P; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) lds_step(k, j);
  }
  __syncthreads();
  // Runs of equal top key bits are in index order; put each in (key, index) order.
  for (int i = threadIdx.x; i < n; i += kBatchSortThreads) {
    const uint32_t h = (uint32_t)(sw[i] >> 32);
    const bool start = i == 0 || (uint32_t)(sw[i - 1] >> 32) != h;
    if (!start || i + 1 >= n || (uint32_t)(sw[i + 1] >> 32) != h) continue;
    int e = i + 2;
    while (e < n && (uint32_t)(sw[e] >> 32) == h) ++e;
    for (int a = i + 1; a < e; ++a) {  // insertion sort of the run [i, e)
      const uint64_t x = sw[a];
      const uint64_t kx = mink2_key(skey, (uint32_t)x);
      int b = a - 1;
      for (; b >= i; --b) {
        const uint64_t kb = mink2_key(skey, (uint32_t)sw[b]);
        if (kb < kx || (kb == kx && (uint32_t)sw[b] < (uint32_t)x)) break;
        sw[b + 1] = sw[b];
      }
      sw[b + 1] = x;
    }
  }
  __syncthreads();
  double* cu = coords + d.coord_off;
  double* cv = cu + n;
  for (int i = threadIdx.x; i < n; i += kBatchSortThreads) {
    const uint64_t g = (uint32_t)sw[i];
    cu[i] = (double)(sm_output(skey, 2 * g) >> 11) * 0x1.0p-53;
    cv[i] = (double)(sm_output(skey, 2 * g + 1) >> 11) * 0x1.0p-53;
  }
}

}  // namespace

size_t sprinkle_ws_bytes(int region, int64_t n) { return layout(region, n, nullptr, nullptr); }

cs_status launch_sprinkle(int region, double eta0, uint64_t seed, int64_t n, double* coords,
                          void* ws, hipStream_t st) {
  SprinkleWs w;
  layout(region, n, ws, &w);
  const int64_t P = pow2_at_least(n);
  const int planes = coord_planes(region);
  const unsigned gridP = (unsigned)ceil_div(P, kBlock);
  if (region == CS_MINK2_DIAMOND && n <= kRankMaxN) {
    hipLaunchKernelGGL(k_rank_place_mink2, dim3((unsigned)ceil_div(n, kRankPer)), dim3(kRankThreads),
                       0, st, sm_stream_key(seed, kStreamMink2), n, coords);
    CS_LAUNCH_CHECK();
    return CS_OK;
  }
  if (region == CS_MINK2_DIAMOND) {
    hipLaunchKernelGGL(k_sprinkle_mink2, dim3(gridP), dim3(kBlock), 0, st,
                       sm_stream_key(seed, kStreamMink2), n, P, w.raw, w.keys, w.gens);
    CS_LAUNCH_CHECK();
  } else if (is_rejection(region)) {
    const bool d4 = region == CS_MINK4_DIAMOND;
    const int64_t M = mink_candidates(region, n);
    const int64_t nblk = M / kBlock;
    const uint64_t skey = sm_stream_key(seed, d4 ? kStreamMink4 : kStreamMink3);
    if (d4) hipLaunchKernelGGL(k_mink_count<4>, dim3((unsigned)nblk), dim3(kBlock), 0, st, skey,
                               w.blk_count);
    else hipLaunchKernelGGL(k_mink_count<3>, dim3((unsigned)nblk), dim3(kBlock), 0, st, skey,
                            w.blk_count);
    CS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, w.blk_count, nblk, w.blk_offset);
    CS_LAUNCH_CHECK();
    if (d4) hipLaunchKernelGGL(k_mink_scatter<4>, dim3((unsigned)nblk), dim3(kBlock), 0, st, skey,
                               n, w.blk_offset, w.raw, w.keys, w.gens);
    else hipLaunchKernelGGL(k_mink_scatter<3>, dim3((unsigned)nblk), dim3(kBlock), 0, st, skey,
                            n, w.blk_offset, w.raw, w.keys, w.gens);
    CS_LAUNCH_CHECK();
    if (d4) hipLaunchKernelGGL(k_mink_tail<4>, dim3(1), dim3(kBlock), 0, st, skey, n, M,
                               w.blk_offset + nblk, w.raw, w.keys, w.gens);
    else hipLaunchKernelGGL(k_mink_tail<3>, dim3(1), dim3(kBlock), 0, st, skey, n, M,
                            w.blk_offset + nblk, w.raw, w.keys, w.gens);
    CS_LAUNCH_CHECK();
    if (P > n) {
      hipLaunchKernelGGL(k_pad_keys, dim3((unsigned)ceil_div(P - n, kBlock)), dim3(kBlock), 0, st,
                         n, P, w.keys, w.gens);
      CS_LAUNCH_CHECK();
    }
  } else if (region == CS_DS2_SLAB) {
    hipLaunchKernelGGL(k_sprinkle_ds2, dim3(gridP), dim3(kBlock), 0, st,
                       sm_stream_key(seed, kStreamDs2), tan(eta0), n, P, w.raw, w.keys, w.gens);
    CS_LAUNCH_CHECK();
  } else {
    hipLaunchKernelGGL(k_sprinkle_ds4, dim3(gridP), dim3(kBlock), 0, st,
                       sm_stream_key(seed, kStreamDsTime), sm_stream_key(seed, kStreamDsSphere),
                       tan(eta0), n, P, w.raw, w.keys, w.gens);
    CS_LAUNCH_CHECK();
  }
  if (n <= kRankMaxN) {
    hipLaunchKernelGGL(k_rank_place, dim3((unsigned)ceil_div(n, kRankPer)), dim3(kRankThreads), 0,
                       st, w.keys, w.raw, planes, n, coords);
    CS_LAUNCH_CHECK();
    return CS_OK;
  }
  cs_status s = bitonic_sort(w.keys, w.gens, P, st);
  if (s != CS_OK) return s;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, st, w.raw,
                     w.gens, planes, n, coords);
  CS_LAUNCH_CHECK();
  return CS_OK;
}

cs_status launch_sprinkle_batch(const uint64_t* seeds, const BatchInst* inst, int64_t count,
                                double* coords, uint64_t* hist, uint64_t* zero, int nzero,
                                hipStream_t st) {
  if (count <= 0) return CS_OK;
  hipLaunchKernelGGL(k_sprinkle_mink2_batch, dim3((unsigned)count), dim3(kBatchSortThreads), 0, st,
                     seeds, inst, coords, hist, zero, nzero);
  CS_LAUNCH_CHECK();
  return CS_OK;
}

}  // namespace cs
