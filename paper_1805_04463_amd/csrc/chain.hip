// Longest chains inside Alexandroff sets (Sec. 2.5.2 "Set Partitions", algorithm "Maximal
// Chain Length") and the degree vectors of the causal matrix (Sec. 3.2).
//
// The algorithm walks an Alexandroff set A_ij recursively with a memo of distances.  A
// recursion is a poor fit for 64-wide wavefronts, so the same quantity is computed
// through Mirsky's theorem instead: in a finite order, the elements whose longest chain
// (counted from below) has h elements are exactly those removed in round h when minimal
// elements are removed repeatedly.  For the set X = A_ij ∪ {j}, round h removes the
// elements h links above i, and j goes last: the number of rounds is the number of links
// of the longest chain from i to j.
//
// Each round tests, for every element k still in X, whether any element of its past is
// still in X.  Each k keeps a witness: the latest past element still in X that a scan of
// its row, from k downward, last found.  Words above the witness's word were seen empty
// (of remaining elements) and stay empty, because X only shrinks.  A round is two
// launches; the first has one wavefront per 64-element word of X (blockIdx.y = the pair):
//   - R_t[w] (the members left) is formed from R_{t-1} and last round's removals P_{t-1};
//   - a member whose witness is not in P_{t-1} is done without touching the matrix;
//   - otherwise its lane reads the next four words of its row, from the witness's word
//     down: a hit gives the new witness (the latest element in the word), and a member
//     with no word left below is removed;
//   - the members with a longer row left are queued (64 sub-queues, one counter add per
//     wave); a second launch gives each of them a wavefront, which scans 64 words, then
//     256, then 1024 words per step (16 coalesced loads per lane), and records the next
//     witness or removes the member.  The graded steps keep a witness found near the
//     top (the common case, e.g. every first witness of round 0) from paying a full
//     1024-word fetch.
// The first launch's wave owns R_t[w] and P_t[w] (the second only sets bits of queued
// members in P_t, with atomicOr).  Over all rounds every
// row word is read about once.  Membership and removals are double-buffered by round
// parity; per pair the rows of R and P have W = ceil(n/64) words.  A member without a
// witness holds -(resume word) - 1 instead.  The host launches rounds in batches; after
// each batch one small launch counts the members left.
#include <math.h>

#include <algorithm>
#include <vector>

#include "common.h"

namespace cs {
namespace {

constexpr int kChainBlock = 256;  // four wavefronts
constexpr int kChainWaves = kChainBlock / kWave;
constexpr int kNear = 4;          // words from a lost witness down that each lane tries
constexpr int kScanMid = 4;       // 64-word loads of the second scan step
constexpr int kScanDepth = 16;    // 64-word loads in flight per wave in a long scan step
constexpr int kLeftBlocks = 256;  // blocks of the "members left" count
constexpr int kQueues = 64;       // long-scan sub-queues (spreads the counter adds)
constexpr int kScanBlocksPerQueue = 32;  // 128 wavefronts per sub-queue

__device__ __forceinline__ uint64_t below_mask(int lane) {
  return lane ? (~0ull >> (kWave - lane)) : 0ull;
}

// R_0, written into R[1] where round 0 reads it as "R_{-1}" (with P_{-1} = P[1] = 0):
// X = {k : lo ≺ k and (k ≺ hi or k = hi)}, lo = -1 / hi = n being the virtual elements
// below / above everything.  No member has a witness yet: each resumes at its own word.
__global__ __launch_bounds__(kChainBlock) void k_chain_init(
    const uint64_t* __restrict__ bits, int64_t n, int64_t ld, int64_t W,
    const int32_t* __restrict__ lohi, uint64_t* __restrict__ R1, uint64_t* __restrict__ P1,
    int32_t* __restrict__ wit, int32_t* __restrict__ height, int32_t* __restrict__ maxh) {
  const int s = blockIdx.y;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t w = (int64_t)blockIdx.x * kChainWaves + (threadIdx.x >> 6);
  if (blockIdx.x == 0 && threadIdx.x == 0) maxh[s] = 0;
  if (w >= W) return;
  const int64_t lo = lohi[2 * s], hi = lohi[2 * s + 1];
  const int64_t k = w * kWave + lane;
  bool in = k < n && k > lo && k <= hi;
  if (in && lo >= 0) in = (bits[lo * ld + w] >> lane) & 1;              // lo ≺ k
  if (in && hi < n && k < hi) in = (bits[hi * ld + w] >> lane) & 1;     // k ≺ hi
  const uint64_t word = __ballot(in);
  if (lane == 0) {
    R1[(int64_t)s * W + w] = word;
    P1[(int64_t)s * W + w] = 0;
  }
  if (k < n) {
    wit[(int64_t)s * n + k] = (int32_t)(-w - 1);
    height[(int64_t)s * n + k] = 0;
  }
}

// Round t.  Rp/Pp: R_{t-1} and P_{t-1}; Rt/Pt: this round's buffers.
__global__ __launch_bounds__(kChainBlock) void k_chain_round(
    const uint64_t* __restrict__ bits, int64_t n, int64_t ld, int64_t W,
    const int32_t* __restrict__ lohi, const uint64_t* __restrict__ Rp,
    const uint64_t* __restrict__ Pp, uint64_t* __restrict__ Rt, uint64_t* __restrict__ Pt,
    int32_t* __restrict__ wit, int32_t* __restrict__ height,
    unsigned long long* __restrict__ qcount, uint64_t* __restrict__ queue, int64_t qcap,
    int32_t t) {
  const int s = blockIdx.y;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t w = (int64_t)blockIdx.x * kChainWaves + (threadIdx.x >> 6);
  if (w >= W) return;
  const int64_t base = (int64_t)s * W;
  const uint64_t* rp = Rp + base;
  const uint64_t* pp = Pp + base;
  const uint64_t rw = rp[w] & ~pp[w];  // R_t[w]
  if (lane == 0) Rt[base + w] = rw;
  if (rw == 0) return;
  const int64_t lo = lohi[2 * s];
  const int64_t wlo = lo < 0 ? 0 : (lo + 1) >> 6;  // no member of X lies below this word
  const int64_t k = w * kWave + lane;
  int32_t* wk = wit + (int64_t)s * n + k;
  bool gone = false, longscan = false;
  int64_t resume = 0;
  if ((rw >> lane) & 1) {
    const int32_t m = *wk;
    if (m < 0 || ((pp[m >> 6] >> (m & 63)) & 1)) {  // no witness, or removed last round
      const int64_t r = m >= 0 ? (int64_t)(m >> 6) : (int64_t)(-m - 1);
      const uint64_t* row = bits + k * ld;
      uint64_t v[kNear];
#pragma unroll
      for (int j = 0; j < kNear; ++j) {  // words r, r-1, ..., all loaded at once
        const int64_t q = r - j;
        uint64_t x = q >= wlo ? (row[q] & rp[q] & ~pp[q]) : 0ull;
        if (q == w) x &= below_mask(lane);  // own word: the past only
        v[j] = x;
      }
      int32_t nm = -1;
#pragma unroll
      for (int j = kNear - 1; j >= 0; --j)
        if (v[j]) nm = (int32_t)((r - j) * kWave + 63 - __builtin_clzll(v[j]));
      if (nm >= 0) {
        *wk = nm;
      } else if (r - kNear >= wlo) {
        longscan = true;  // words r-kNear+1 .. r hold none: go on from r-kNear
        resume = r - kNear;
      } else {
        gone = true;  // no member of its past is left: k is minimal in R_t
      }
    }
  }
  const uint64_t removed = __ballot(gone);
  if (gone) height[(int64_t)s * n + k] = t + 1;
  if (lane == 0) Pt[base + w] = removed;  // the scan launch adds the queued members' bits
  // Longer rows go to one of kQueues sub-queues (by block), one counter add per wave.
  const uint64_t todo = __ballot(longscan);
  if (todo == 0) return;
  if (longscan) wit[(int64_t)s * n + k] = (int32_t)(-resume - 1);
  const int64_t blk = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  const int g = (int)(blk % kQueues);
  unsigned long long slot = 0;
  if (lane == 0) slot = atomicAdd(&qcount[g], (unsigned long long)__popcll(todo));
  slot = __shfl(slot, 0);
  if (longscan) {
    const uint64_t rank = __popcll(todo & ((1ull << lane) - 1));
    queue[(int64_t)g * qcap + (int64_t)slot + rank] = ((uint64_t)s << 32) | (uint64_t)k;
  }
}

// Highest word q in [wlo, top] of row k holding a member of R_t, looking at J * 64 words
// (lane l, load j: word top - l - 64 j); -1 if none of them has one.  top lies below k's
// own word, so no bit needs masking.
template <int J>
__device__ __forceinline__ int64_t scan_step(const uint64_t* __restrict__ row,
                                             const uint64_t* __restrict__ R, int64_t top,
                                             int64_t wlo, int lane) {
  uint64_t v[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int64_t q = top - lane - (int64_t)kWave * j;
    v[j] = q >= wlo ? (row[q] & R[q]) : 0ull;
  }
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const uint64_t hit = __ballot(v[j] != 0);
    if (hit) return top - (int64_t)__builtin_ctzll(hit) - (int64_t)kWave * j;
  }
  return -1;
}

// Round t, second half: one wavefront per queued member; blockIdx.y = the sub-queue.  Also
// clears the counters the next round will fill (last read by the previous round).
__global__ __launch_bounds__(kChainBlock) void k_chain_scan(
    const uint64_t* __restrict__ bits, int64_t n, int64_t ld, int64_t W,
    const int32_t* __restrict__ lohi, const uint64_t* __restrict__ Rt, uint64_t* __restrict__ Pt,
    int32_t* __restrict__ wit, int32_t* __restrict__ height,
    const unsigned long long* __restrict__ qcount, unsigned long long* __restrict__ qnext,
    const uint64_t* __restrict__ queue, int64_t qcap, int32_t t) {
  const int lane = threadIdx.x & (kWave - 1);
  const int g = blockIdx.y;
  if (blockIdx.x == 0 && threadIdx.x == 0) qnext[g] = 0;
  const int64_t gw = (int64_t)blockIdx.x * kChainWaves + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * kChainWaves;
  const int64_t items = (int64_t)qcount[g];
  const uint64_t* q = queue + (int64_t)g * qcap;
  for (int64_t i = gw; i < items; i += nw) {
    const uint64_t item = q[i];
    const int s = (int)(item >> 32);
    const int64_t k = (int64_t)(item & 0xffffffffull);
    const int64_t lo = lohi[2 * s];
    const int64_t wlo = lo < 0 ? 0 : (lo + 1) >> 6;
    const int64_t base = (int64_t)s * W;
    const uint64_t* R = Rt + base;
    const uint64_t* row = bits + k * ld;
    int32_t* wk = wit + (int64_t)s * n + k;
    int64_t top = -(int64_t)(*wk) - 1;  // resume word, below k's own word
    int64_t found = scan_step<1>(row, R, top, wlo, lane);  // a witness nearby is common
    top -= kWave;
    if (found < 0 && top >= wlo) {  // then 256 words before the 1024-word steps
      found = scan_step<kScanMid>(row, R, top, wlo, lane);
      top -= (int64_t)kWave * kScanMid;
    }
    while (found < 0 && top >= wlo) {
      found = scan_step<kScanDepth>(row, R, top, wlo, lane);
      top -= (int64_t)kWave * kScanDepth;
    }
    if (lane == 0) {
      if (found >= 0) {
        *wk = (int32_t)(found * kWave + 63 - __builtin_clzll(row[found] & R[found]));
      } else {
        height[(int64_t)s * n + k] = t + 1;
        atomicOr(&Pt[base + (k >> 6)], 1ull << (k & 63));
      }
    }
  }
}

// count += the members left after a round, the bits of R & ~P (that round's membership and
// removals); one counter add per block.
__global__ __launch_bounds__(kChainBlock) void k_chain_left(const uint64_t* __restrict__ R,
                                                           const uint64_t* __restrict__ P,
                                                           int64_t words,
                                                           unsigned long long* __restrict__ count) {
  __shared__ unsigned long long part[kChainWaves];
  unsigned long long mine = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    mine += __popcll(R[i] & ~P[i]);
  for (int off = kWave / 2; off > 0; off >>= 1) mine += __shfl_xor(mine, off);
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x >> 6] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kChainWaves; ++i) mine += part[i];
    if (mine) atomicAdd(count, mine);
  }
}

// maxh[s] = the largest height of pair s (pairs ending at the virtual top only); blocks of
// blockIdx.x split the n heights, one atomicMax each.
__global__ __launch_bounds__(kChainBlock) void k_chain_maxh(const int32_t* __restrict__ lohi,
                                                           const int32_t* __restrict__ height,
                                                           int64_t n, int32_t* __restrict__ maxh) {
  const int s = blockIdx.y;
  if (lohi[2 * s + 1] != n) return;
  const int32_t* h = height + (int64_t)s * n;
  __shared__ int32_t part[kChainWaves];
  int32_t mx = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    mx = max(mx, h[k]);
  for (int off = kWave / 2; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off));
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kChainWaves; ++i) mx = max(mx, part[i]);
    if (mx) atomicMax(&maxh[s], mx);
  }
}

// length[s]: the height of hi (0 when hi is not in X, i.e. lo does not precede it), or,
// for the virtual top, one link above the highest element.
__global__ void k_chain_length(const int32_t* __restrict__ lohi, const int32_t* __restrict__ height,
                               const int32_t* __restrict__ maxh, int64_t count, int64_t n,
                               int32_t* __restrict__ length) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= count) return;
  const int64_t hi = lohi[2 * s + 1];
  length[s] = hi < n ? height[s * n + hi] : maxh[s] + 1;
}

// Degree vectors: one wavefront per row, 128 words per step (16-byte loads).
__global__ __launch_bounds__(kChainBlock) void k_degrees(const uint64_t* __restrict__ bits,
                                                        int64_t n, int64_t ld, int64_t W,
                                                        int64_t* __restrict__ indeg,
                                                        int64_t* __restrict__ outdeg) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t k = (int64_t)blockIdx.x * kChainWaves + (threadIdx.x >> 6);
  if (k >= n) return;
  const uint64_t* row = bits + k * ld;
  const int64_t kw = k >> 6;
  const uint64_t below = (k & 63) ? (~0ull >> (64 - (k & 63))) : 0ull;
  const uint64_t tail = (n & 63) ? (~0ull >> (64 - (n & 63))) : ~0ull;
  uint32_t cin = 0, cout = 0;
  for (int64_t w0 = 2 * lane; w0 < W; w0 += 2 * kWave) {
    const ulonglong2 v2 = *reinterpret_cast<const ulonglong2*>(row + w0);  // W <= ld, ld even
    uint64_t v[2] = {v2.x, v2.y};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t w = w0 + j;
      if (w >= W) break;
      uint64_t x = v[j];
      if (w == W - 1) x &= tail;
      if (w < kw) {
        cin += __popcll(x);
      } else if (w > kw) {
        cout += __popcll(x);
      } else {
        cin += __popcll(x & below);
        cout += __popcll(x & ~below & ~(1ull << (k & 63)));
      }
    }
  }
  for (int off = kWave / 2; off > 0; off >>= 1) {
    cin += __shfl_xor(cin, off);
    cout += __shfl_xor(cout, off);
  }
  if (lane == 0) {
    if (indeg) indeg[k] = cin;
    if (outdeg) outdeg[k] = cout;
  }
}

struct ChainWs {
  int32_t* lohi;
  unsigned long long* left;   // members left: before round 0, then after each batch
  int32_t* maxh;
  uint64_t* R[2];
  uint64_t* P[2];
  int32_t* wit;
  int32_t* height;  // used when the caller passes none
  unsigned long long* qcount[2];  // kQueues counters per round parity
  uint64_t* queue;                // kQueues sub-queues of qcap items
  int64_t qcap;
  size_t bytes;
};

int64_t max_batches(int64_t n) { return n / 2 + 2; }  // every batch has at least 2 rounds

ChainWs chain_layout(void* base, int64_t n, int64_t count) {
  const int64_t W = ceil_div(n, kWave);
  ChainWs L{};
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off = align_up(off + b, 256);
    return (char*)base + o;
  };
  L.lohi = (int32_t*)take(sizeof(int32_t) * 2 * count);
  L.left = (unsigned long long*)take(sizeof(unsigned long long) * (max_batches(n) + 1));
  L.maxh = (int32_t*)take(sizeof(int32_t) * count);
  for (int b = 0; b < 2; ++b) {
    L.R[b] = (uint64_t*)take(sizeof(uint64_t) * W * count);
    L.P[b] = (uint64_t*)take(sizeof(uint64_t) * W * count);
  }
  L.wit = (int32_t*)take(sizeof(int32_t) * n * count);
  L.height = (int32_t*)take(sizeof(int32_t) * n * count);
  for (int b = 0; b < 2; ++b)
    L.qcount[b] = (unsigned long long*)take(sizeof(unsigned long long) * kQueues);
  // sub-queue g takes the members of the round launch's blocks numbered g mod kQueues
  const int64_t blocks = ceil_div(W, kChainWaves) * count;
  L.qcap = ceil_div(blocks, kQueues) * kChainBlock;
  L.queue = (uint64_t*)take(sizeof(uint64_t) * L.qcap * kQueues);
  L.bytes = off;
  return L;
}

}  // namespace

size_t chain_ws_bytes(int64_t n, int64_t count) {
  return chain_layout(nullptr, n, count).bytes;
}

cs_status launch_longest_chain(const uint64_t* bits, int64_t n, int64_t ld, const int64_t* lo,
                               const int64_t* hi, int64_t count, int32_t* length,
                               int32_t* height, void* ws, hipStream_t st) {
  ChainWs L = chain_layout(ws, n, count);
  int32_t* h = height ? height : L.height;
  const int64_t W = ceil_div(n, kWave);
  std::vector<int32_t> lohi(2 * count);
  for (int64_t s = 0; s < count; ++s) {
    lohi[2 * s] = (int32_t)lo[s];
    lohi[2 * s + 1] = (int32_t)hi[s];
  }
  CS_HIP_CHECK(hipMemcpyAsync(L.lohi, lohi.data(), sizeof(int32_t) * 2 * count,
                              hipMemcpyHostToDevice, st));
  cs_status s0 = launch_fill_u64((uint64_t*)L.left, max_batches(n) + 1, 0, st);
  if (s0 == CS_OK) s0 = launch_fill_u64((uint64_t*)L.qcount[0], kQueues, 0, st);
  if (s0 == CS_OK) s0 = launch_fill_u64((uint64_t*)L.qcount[1], kQueues, 0, st);
  if (s0 != CS_OK) return s0;
  const dim3 grid((unsigned)ceil_div(W, kChainWaves), (unsigned)count);
  hipLaunchKernelGGL(k_chain_init, grid, dim3(kChainBlock), 0, st, bits, n, ld, W, L.lohi, L.R[1],
                     L.P[1], L.wit, h, L.maxh);
  CS_LAUNCH_CHECK();
  const int64_t words = W * count;
  const dim3 red((unsigned)std::min<int64_t>(kLeftBlocks, ceil_div(words, kChainBlock)));
  hipLaunchKernelGGL(k_chain_left, red, dim3(kChainBlock), 0, st, L.R[1], L.P[1], words, L.left);
  CS_LAUNCH_CHECK();
  // Round t removes the minimal elements of R_t; every X is empty after at most n rounds.
  // Batches of rounds end with a count of the members left; the next batch is sized from
  // the rate of removal so far, so that few rounds run past the end.
  int64_t t = 0, batch = 8, b = 0;
  unsigned long long counts[2] = {0, 1};
  while (t <= n && b < max_batches(n)) {
    const int64_t end = std::min<int64_t>(t + batch, n + 1);
    for (; t < end; ++t) {
      const int c = (int)(t & 1), p = c ^ 1;
      hipLaunchKernelGGL(k_chain_round, grid, dim3(kChainBlock), 0, st, bits, n, ld, W, L.lohi,
                         L.R[p], L.P[p], L.R[c], L.P[c], L.wit, h, L.qcount[c], L.queue, L.qcap,
                         (int32_t)t);
      CS_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_chain_scan, dim3(kScanBlocksPerQueue, kQueues), dim3(kChainBlock), 0,
                         st, bits, n, ld, W, L.lohi, L.R[c], L.P[c], L.wit, h,
                         L.qcount[c], L.qcount[p], L.queue, L.qcap, (int32_t)t);
      CS_LAUNCH_CHECK();
    }
    ++b;  // members left after round t-1: R_{t-1} & ~P_{t-1}
    hipLaunchKernelGGL(k_chain_left, red, dim3(kChainBlock), 0, st, L.R[(t - 1) & 1],
                       L.P[(t - 1) & 1], words, L.left + b);
    CS_LAUNCH_CHECK();
    CS_HIP_CHECK(hipMemcpyAsync(counts, L.left + b - 1, sizeof(counts), hipMemcpyDeviceToHost, st));
    CS_HIP_CHECK(hipStreamSynchronize(st));
    if (counts[1] == 0) break;
    const double rate = (double)(counts[0] - counts[1]) / (double)batch;  // >= 1 per round
    // Layers thin out towards the end, so the rate so far under-estimates the rounds
    // left; half again as many rounds (a round past the end is two near-empty launches)
    // saves host round trips: 1.76 -> 1.62 ms on the whole 3+1 order at N = 131072.
    const int64_t want = (int64_t)ceil(1.5 * (double)counts[1] / rate);
    batch = std::max<int64_t>(2, std::min<int64_t>(64, want));
  }
  if (counts[1] != 0) return CS_ERR_HIP;  // unreachable for a valid order
  hipLaunchKernelGGL(k_chain_maxh, dim3((unsigned)std::min<int64_t>(64, ceil_div(n, 4096)),
                                        (unsigned)count),
                     dim3(kChainBlock), 0, st, L.lohi, h, n, L.maxh);
  CS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_chain_length, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, st,
                     L.lohi, h, L.maxh, count, n, length);
  CS_LAUNCH_CHECK();
  return CS_OK;
}

cs_status launch_degrees(const uint64_t* bits, int64_t n, int64_t ld, int64_t* indeg,
                         int64_t* outdeg, hipStream_t st) {
  const int64_t W = ceil_div(n, kWave);
  hipLaunchKernelGGL(k_degrees, dim3((unsigned)ceil_div(n, kChainWaves)), dim3(kChainBlock), 0,
                     st, bits, n, ld, W, indeg, outdeg);
  CS_LAUNCH_CHECK();
  return CS_OK;
}

}  // namespace cs
