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
// still in X.  Each k keeps a witness pointer: the word of its row where a past element
// still in X was last found, scanning from k downward.  Words above the pointer were seen
// empty (of remaining elements) and stay empty, because X only shrinks; so a round first
// re-checks the one witness word, and only when that element has gone does the wave scan
// further down, 256 words per step.  Over all rounds every row word is read about once.
//
// Layout: one wavefront per 64-element word of X (the membership bitset), a block of
// four wavefronts, blockIdx.y = the pair (its membership row has W = ceil(n/64) words).
// Membership is double-buffered: round t reads
// R_t and writes R_{t+1}, each wave its own word, so a round needs no atomics on it.  The
// host launches rounds in batches and reads back a per-round count of non-empty words
// to stop.
#include <algorithm>
#include <vector>

#include "common.h"

namespace cs {
namespace {

constexpr int kChainBlock = 256;            // four wavefronts, four words of X
constexpr int kChainWaves = kChainBlock / kWave;
constexpr int kScanPerLane = 4;             // words per lane per scan step

__device__ inline uint64_t wave_ballot(bool p) { return __ballot(p); }

// R_0: X = {k : lo ≺ k and (k ≺ hi or k = hi)}, with lo = -1 / hi = n as the virtual
// elements below / above everything.  Witness pointers start at the element's own word.
__global__ __launch_bounds__(kChainBlock) void k_chain_init(
    const uint64_t* __restrict__ bits, int64_t n, int64_t ld, int64_t W,
    const int32_t* __restrict__ lohi, uint64_t* __restrict__ R0, int32_t* __restrict__ ptr,
    int32_t* __restrict__ height, int32_t* __restrict__ layers) {
  const int s = blockIdx.y;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t w = (int64_t)blockIdx.x * kChainWaves + (threadIdx.x >> 6);
  if (blockIdx.x == 0 && threadIdx.x == 0) layers[s] = 0;
  if (w >= W) return;
  const int64_t lo = lohi[2 * s], hi = lohi[2 * s + 1];
  const int64_t k = w * kWave + lane;
  bool in = k < n && k > lo && k <= hi;
  if (in && lo >= 0) in = (bits[lo * ld + w] >> lane) & 1;              // lo ≺ k
  if (in && hi < n && k < hi) in = (bits[hi * ld + w] >> lane) & 1;     // k ≺ hi
  const uint64_t word = wave_ballot(in);
  if (lane == 0) R0[(int64_t)s * W + w] = word;
  if (k < n) {
    ptr[(int64_t)s * n + k] = (int32_t)w;
    if (height) height[(int64_t)s * n + k] = 0;
  }
}

// Round t: remove the minimal elements of R_t, the elements t+1 links above lo.
__global__ __launch_bounds__(kChainBlock) void k_chain_step(
    const uint64_t* __restrict__ bits, int64_t n, int64_t ld, int64_t W,
    const int32_t* __restrict__ lohi, const uint64_t* __restrict__ Rc, uint64_t* __restrict__ Rn,
    int32_t* __restrict__ ptr, int32_t* __restrict__ height, int32_t* __restrict__ layers,
    unsigned long long* __restrict__ alive, int32_t t) {
  const int s = blockIdx.y;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t w = (int64_t)blockIdx.x * kChainWaves + (threadIdx.x >> 6);
  if (w >= W) return;
  const uint64_t* R = Rc + (int64_t)s * W;
  const uint64_t rw = R[w];
  if (rw == 0) {
    if (lane == 0) Rn[(int64_t)s * W + w] = 0;
    return;
  }
  const int64_t lo = lohi[2 * s];
  const int64_t wlo = lo < 0 ? 0 : (lo + 1) >> 6;  // no element of X lies below this word
  const int64_t k = w * kWave + lane;
  const bool in = (rw >> lane) & 1;

  // Re-check the witness word (in its own word, only the bits below k are its past).
  int32_t p = 0;
  bool ok = false;
  if (in) {
    p = ptr[(int64_t)s * n + k];
    uint64_t x = bits[k * ld + p] & R[p];
    if (p == w) x &= lane ? (~0ull >> (kWave - lane)) : 0ull;
    ok = x != 0;
  }

  // Elements whose witness has gone: the wave scans each one's row further down.
  uint64_t need = wave_ballot(in && !ok);
  int32_t np = p;
  while (need) {
    const int e = __builtin_ctzll(need);
    need &= need - 1;
    const int64_t ke = w * kWave + e;
    const uint64_t* row = bits + ke * ld;
    const int32_t pe = __builtin_amdgcn_readlane(p, e);
    int32_t found = -1;
    for (int64_t top = (int64_t)pe - 1; top >= wlo; top -= kWave * kScanPerLane) {
      const int64_t q0 = top - (int64_t)kScanPerLane * lane;
      uint64_t v[kScanPerLane];
#pragma unroll
      for (int j = 0; j < kScanPerLane; ++j) {
        const int64_t q = q0 - j;
        v[j] = q >= wlo ? (row[q] & R[q]) : 0ull;
      }
      int32_t best = -1;
#pragma unroll
      for (int j = kScanPerLane - 1; j >= 0; --j)
        if (v[j]) best = (int32_t)(q0 - j);  // the highest word with a hit wins
      const uint64_t hit = wave_ballot(best >= 0);
      if (hit) {
        found = __builtin_amdgcn_readlane(best, (int)__builtin_ctzll(hit));
        break;
      }
    }
    if (lane == e) np = found;
  }

  const bool peel = in && np < 0;
  const uint64_t gone = wave_ballot(peel);
  if (in && !ok && np >= 0) ptr[(int64_t)s * n + k] = np;
  if (peel && height) height[(int64_t)s * n + k] = t + 1;
  const uint64_t next = rw & ~gone;
  if (lane == 0) {
    Rn[(int64_t)s * W + w] = next;
    atomicMax(&layers[s], t + 1);
    if (next) atomicAdd(&alive[t], 1ull);
  }
}

__global__ void k_chain_finish(const int32_t* __restrict__ lohi, const int32_t* __restrict__ layers,
                               int64_t count, int64_t n, int32_t* __restrict__ length) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= count) return;
  // the virtual top is one link above the last round's elements
  length[s] = layers[s] + (lohi[2 * s + 1] == n ? 1 : 0);
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
  int32_t* layers;
  unsigned long long* alive;
  uint64_t* R[2];
  int32_t* ptr;
  size_t bytes;
};

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
  L.layers = (int32_t*)take(sizeof(int32_t) * count);
  L.alive = (unsigned long long*)take(sizeof(unsigned long long) * n);
  L.R[0] = (uint64_t*)take(sizeof(uint64_t) * W * count);
  L.R[1] = (uint64_t*)take(sizeof(uint64_t) * W * count);
  L.ptr = (int32_t*)take(sizeof(int32_t) * n * count);
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
  const int64_t W = ceil_div(n, kWave);
  std::vector<int32_t> lohi(2 * count);
  for (int64_t s = 0; s < count; ++s) {
    lohi[2 * s] = (int32_t)lo[s];
    lohi[2 * s + 1] = (int32_t)hi[s];
  }
  CS_HIP_CHECK(hipMemcpyAsync(L.lohi, lohi.data(), sizeof(int32_t) * 2 * count,
                              hipMemcpyHostToDevice, st));
  cs_status s0 = launch_fill_u64((uint64_t*)L.alive, n, 0, st);
  if (s0 != CS_OK) return s0;
  const dim3 grid((unsigned)ceil_div(W, kChainWaves), (unsigned)count);
  hipLaunchKernelGGL(k_chain_init, grid, dim3(kChainBlock), 0, st, bits, n, ld, W, L.lohi, L.R[0],
                     L.ptr, height, L.layers);
  CS_LAUNCH_CHECK();
  // At most |X| <= n rounds: every round of a non-empty X removes its minimal elements.
  int64_t t = 0, batch = 4;
  unsigned long long left = 1;
  while (t < n) {
    const int64_t end = std::min<int64_t>(t + batch, n);
    for (; t < end; ++t) {
      hipLaunchKernelGGL(k_chain_step, grid, dim3(kChainBlock), 0, st, bits, n, ld, W, L.lohi,
                         L.R[t & 1], L.R[(t + 1) & 1], L.ptr, height, L.layers, L.alive,
                         (int32_t)t);
      CS_LAUNCH_CHECK();
    }
    CS_HIP_CHECK(hipMemcpyAsync(&left, L.alive + (t - 1), sizeof(left), hipMemcpyDeviceToHost, st));
    CS_HIP_CHECK(hipStreamSynchronize(st));
    if (left == 0) break;
    batch = std::min<int64_t>(2 * batch, 64);
  }
  if (left != 0) return CS_ERR_HIP;  // unreachable for a valid order
  hipLaunchKernelGGL(k_chain_finish, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, st,
                     L.lohi, L.layers, count, n, length);
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
