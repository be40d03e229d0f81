// Interval counters: N_m = #{i < j : i ≺ j, |{k : i ≺ k ≺ j}| = m}
// (eq. IOIs; algorithms "Naive" and "Optimized Interval Abundance Measurement").
//
// For a related pair the interval size is the inner product of row i and row j of
// the symmetric bitset S over the columns strictly between i and j (the caption of
// the thesis's figure on order intervals).  With C the strictly upper-triangular
// causal matrix, that is (C.C)_ij = sum_k C_ik C_kj, and both factors are rows of
// S: A = rows of the output-tile rows restricted to k > i, B = rows of the
// output-tile columns restricted to k < j.  So an output tile (I, J) of the
// upper triangle is an "NT" product of two row panels of S over K in [I, J].
//
// Both counters share:
//   - a persistent grid that takes output tiles from an atomic counter, longest
//     K-range first (tiles with the same distance J - I from the diagonal have
//     equal cost);
//   - a whole-tile skip when no pair of the tile is related;
//   - K staged through LDS 256 bits at a time with register prefetch of the next
//     stage; the triangular masks (k > i for A, k < j for B) are applied while
//     staging;
//   - an epilogue that tests the related bit S[j][i] of each output and bins the
//     count into a per-workgroup LDS histogram (16384 uint32 bins) or, beyond it,
//     straight into the global uint64 histogram; LDS bins are flushed at exit.
// They differ in the inner product:
//   MFMA   bits are expanded to int8 0/1 in registers and multiplied on
//          v_mfma_i32_32x32x32_i8 with int32 accumulation (exact: counts < 2^31).
//          Because both operands are rows of S, any permutation of k inside a
//          32-bit word works if applied to A and B alike; the expansion used,
//          byte b of register q = bit (4h + q + 8b) of the word (h = lane >> 5),
//          costs two VALU ops per four bytes.
//   BITSET AND + v_bcnt_u32_b32 on 32-bit words, each thread an 8x8 block of pairs.
#include "common.h"

namespace cs {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;
constexpr int kStageBits = 256;         // K bits per LDS stage
constexpr int kStageWords = kStageBits / 32;
constexpr int kLdsBins = 16384;         // per-workgroup histogram bins (uint32)

// Output tile t (0-based) in longest-first order for a T x T tile triangle:
// e = T-1-(J-I) is the diagonal rank, tiles with the same e are consecutive.
__device__ inline void tile_of(int64_t t, int64_t T, int64_t* I, int64_t* J) {
  int64_t e = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (e * (e + 1) / 2 > t) --e;
  while ((e + 1) * (e + 2) / 2 <= t) ++e;
  *I = t - e * (e + 1) / 2;
  *J = *I + (T - 1 - e);
}

// Keep bits k > g (A side) or k < g (B side) of the 32-bit word covering [kw, kw+32).
__device__ inline uint32_t mask_above(int64_t kw, int64_t g) {
  if (kw > g) return 0xFFFFFFFFu;
  if (kw + 32 <= g + 1) return 0u;
  return 0xFFFFFFFFu << (uint32_t)(g + 1 - kw);
}
__device__ inline uint32_t mask_below(int64_t kw, int64_t g) {
  if (kw + 32 <= g) return 0xFFFFFFFFu;
  if (kw >= g) return 0u;
  return (1u << (uint32_t)(g - kw)) - 1u;
}

// LDS position (in uint32) of the 16-byte half `h` of staged row r: rows are 8
// words; the half index is XOR-swizzled with bit 3 of the row to spread banks.
__device__ inline int lds_pos(int r, int h) { return r * kStageWords + ((h ^ ((r >> 3) & 1)) << 2); }

// Global -> register fetch of K stages for a panel of ROWS rows starting at row0.
// Each thread owns ROWS*2/kThreads 16-byte halves (row r = c/2, half h = c%2); its
// row pointers are set once per tile.  The triangular masks only matter on stages
// that overlap the panel's own diagonal block, so they are applied only there.
template <int ROWS>
struct Stage {
  static constexpr int kPer = ROWS * 2 / kThreads;
  uint4 v[kPer];
  const uint4* p[kPer];

  __device__ inline void init(const uint32_t* __restrict__ S32, int64_t ld32, int64_t row0,
                              int64_t n, int64_t kbit0) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int c = threadIdx.x + q * kThreads;
      const int64_t g = row0 + (c >> 1);
      p[q] = g < n ? (const uint4*)(S32 + g * ld32 + (kbit0 >> 5)) + (c & 1) : nullptr;
    }
  }
  // Stage s covers bits [kb, kb + 256), kb = kbit0 + 256 s.  above: keep k > row (A side),
  // else keep k < row (B side).
  __device__ inline void fetch(int64_t s, int64_t kb, int64_t row_bits, int64_t row0,
                               bool masked, bool above) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int c = threadIdx.x + q * kThreads;
      const int h = c & 1;
      const int64_t kw = kb + h * 128;
      uint4 x = make_uint4(0, 0, 0, 0);
      if (p[q] != nullptr && kw < row_bits) x = p[q][2 * s];
      if (masked) {
        const int64_t g = row0 + (c >> 1);
        if (above) {
          x.x &= mask_above(kw, g);
          x.y &= mask_above(kw + 32, g);
          x.z &= mask_above(kw + 64, g);
          x.w &= mask_above(kw + 96, g);
        } else {
          x.x &= mask_below(kw, g);
          x.y &= mask_below(kw + 32, g);
          x.z &= mask_below(kw + 64, g);
          x.w &= mask_below(kw + 96, g);
        }
      }
      v[q] = x;
    }
  }
  __device__ inline void store(uint32_t* lds) const {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int c = threadIdx.x + q * kThreads;
      *(uint4*)(lds + lds_pos(c >> 1, c & 1)) = v[q];
    }
  }
};

// Counts are at most n-2 by construction; the bound check keeps a histogram write in
// range whatever the inputs.  `tmax` tracks the largest LDS bin this thread touched.
__device__ inline void bin_add(uint32_t* lds_hist, unsigned long long* hist, uint32_t bin,
                               int64_t nbins, uint32_t& tmax) {
  if (bin < (uint32_t)kLdsBins) {
    atomicAdd(lds_hist + bin, 1u);
    tmax = bin > tmax ? bin : tmax;
  } else if ((int64_t)bin < nbins) {
    atomicAdd(hist + bin, 1ull);
  }
}

// Adds the LDS bins [0, max touched] to the global histogram and clears them.
__device__ inline void flush_hist(uint32_t* lds_hist, unsigned long long* hist, int64_t nbins,
                                  uint32_t& tmax, uint32_t* s_max) {
  __syncthreads();
  if (threadIdx.x == 0) *s_max = 0;
  __syncthreads();
  atomicMax(s_max, tmax);
  __syncthreads();
  int64_t lim = (int64_t)*s_max + 1;
  lim = lim < nbins ? lim : nbins;
  lim = lim < kLdsBins ? lim : kLdsBins;
  for (int b = threadIdx.x; b < lim; b += kThreads) {
    uint32_t v = lds_hist[b];
    if (v) {
      atomicAdd(hist + b, (unsigned long long)v);
      lds_hist[b] = 0;
    }
  }
  tmax = 0;
  __syncthreads();
}

// Takes the next work index for the workgroup (one atomic per tile).
__device__ inline int64_t next_tile(unsigned int* counter, int* slot) {
  __syncthreads();
  if (threadIdx.x == 0) *slot = (int)atomicAdd(counter, 1u);
  __syncthreads();
  return *slot;
}

struct TileArgs {
  const uint32_t* S32;        // instance matrix, as 32-bit words
  int64_t ld32;               // row stride in 32-bit words
  int64_t n;                  // points of the instance
  int64_t I0, J0;             // first row / first column of the output tile
  unsigned long long* hist;   // instance histogram (n-1 bins)
};

// ===========================================================================
// MFMA tile.  Workgroup tile BM x BM, four waves in 2x2, each WM x WM blocks of
// 32x32 outputs (WM = 4: 256x256 tile, 128x128 per wave, 256 int32 accumulators).
// Returns false (having done nothing) when no pair of the tile is related.
// ===========================================================================
template <int WM>
__device__ inline bool mfma_tile(const TileArgs& ta, uint32_t* As, uint32_t* Bs,
                                 uint32_t* lds_hist, uint32_t& tmax) {
  constexpr int BM = 2 * WM * 32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int hsel = lane >> 5, l32 = lane & 31;
  const int64_t n = ta.n, I0 = ta.I0, J0 = ta.J0, nbins = n - 1;
  const int64_t rb = I0 + wr * (WM * 32);  // first output row of this wave

  // Related bits S[j][i] for this wave's outputs: word mb of column block nb.
  uint32_t relw[WM][WM];
  bool any = false;
#pragma unroll
  for (int nb = 0; nb < WM; ++nb) {
    const int64_t j = J0 + wc * (WM * 32) + nb * 32 + l32;
#pragma unroll
    for (int mb = 0; mb < WM; ++mb) {
      uint32_t w = 0;
      if (j < n) {
        const int64_t i0 = rb + mb * 32;
        w = ta.S32[j * ta.ld32 + (i0 >> 5)];
        w &= mask_below(i0, j);  // only i < j
      }
      relw[nb][mb] = w;
      any |= (w != 0);
    }
  }
  if (!__syncthreads_or(any)) return false;

  v16i acc[WM][WM];
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WM; ++b) acc[a][b] = (v16i){0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};

  const int64_t kbeg = I0;
  const int64_t kend = (J0 + BM < n ? J0 + BM : n);
  const int64_t nst = ceil_div(kend - kbeg, kStageBits);
  const int64_t row_bits = ta.ld32 * 32;
  Stage<BM> sa, sb;
  sa.init(ta.S32, ta.ld32, I0, n, kbeg);
  sb.init(ta.S32, ta.ld32, J0, n, kbeg);
  sa.fetch(0, kbeg, row_bits, I0, kbeg < I0 + BM, true);
  sb.fetch(0, kbeg, row_bits, J0, kbeg + kStageBits > J0, false);
  for (int64_t s = 0; s < nst; ++s) {
    __syncthreads();
    sa.store(As);
    sb.store(Bs);
    __syncthreads();
    if (s + 1 < nst) {
      const int64_t kb = kbeg + (s + 1) * kStageBits;
      sa.fetch(s + 1, kb, row_bits, I0, kb < I0 + BM, true);
      sb.fetch(s + 1, kb, row_bits, J0, kb + kStageBits > J0, false);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint4 aw[WM], bw[WM];
#pragma unroll
      for (int mb = 0; mb < WM; ++mb)
        aw[mb] = *(const uint4*)(As + lds_pos(wr * WM * 32 + mb * 32 + l32, h));
#pragma unroll
      for (int nb = 0; nb < WM; ++nb)
        bw[nb] = *(const uint4*)(Bs + lds_pos(wc * WM * 32 + nb * 32 + l32, h));
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        v4i af[WM], bf[WM];
        const uint32_t sh = 4u * (uint32_t)hsel;
#pragma unroll
        for (int mb = 0; mb < WM; ++mb) {
          const uint32_t x = w == 0 ? aw[mb].x : w == 1 ? aw[mb].y : w == 2 ? aw[mb].z : aw[mb].w;
          af[mb] = (v4i){(int)((x >> sh) & 0x01010101u), (int)((x >> (sh + 1)) & 0x01010101u),
                         (int)((x >> (sh + 2)) & 0x01010101u), (int)((x >> (sh + 3)) & 0x01010101u)};
        }
#pragma unroll
        for (int nb = 0; nb < WM; ++nb) {
          const uint32_t x = w == 0 ? bw[nb].x : w == 1 ? bw[nb].y : w == 2 ? bw[nb].z : bw[nb].w;
          bf[nb] = (v4i){(int)((x >> sh) & 0x01010101u), (int)((x >> (sh + 1)) & 0x01010101u),
                         (int)((x >> (sh + 2)) & 0x01010101u), (int)((x >> (sh + 3)) & 0x01010101u)};
        }
#pragma unroll
        for (int mb = 0; mb < WM; ++mb)
#pragma unroll
          for (int nb = 0; nb < WM; ++nb)
            acc[mb][nb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[mb], bf[nb], acc[mb][nb], 0, 0, 0);
      }
    }
  }

  // Epilogue.  32x32 accumulator layout: lane holds column (lane & 31) and rows
  // 8*(e/4) + 4*(lane/32) + (e%4) for e = 0..15.
#pragma unroll
  for (int nb = 0; nb < WM; ++nb) {
#pragma unroll
    for (int mb = 0; mb < WM; ++mb) {
      const uint32_t w = relw[nb][mb];
      if (!w) continue;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int il = (e >> 2) * 8 + hsel * 4 + (e & 3);
        if ((w >> il) & 1u) bin_add(lds_hist, ta.hist, (uint32_t)acc[mb][nb][e], nbins, tmax);
      }
    }
  }
  return true;
}

// ===========================================================================
// Bitset tile.  Workgroup tile 128 x 128; thread (ty, tx) = (tid/16, tid%16) owns
// rows 8*ty + a and columns tx + 16*b (a, b = 0..7); a wave whose 32 x 128 pairs
// hold no relation skips the arithmetic (it still helps stage).
// ===========================================================================
constexpr int kBitsetTile = 128;

__device__ inline bool bitset_tile(const TileArgs& ta, uint32_t* As, uint32_t* Bs,
                                   uint32_t* lds_hist, uint32_t& tmax) {
  constexpr int BM = kBitsetTile;
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  const int64_t n = ta.n, I0 = ta.I0, J0 = ta.J0, nbins = n - 1;

  // Related bits: for row i = I0 + 8ty + a, the columns tx + 16b are taken from the
  // row's 128-bit slice over [J0, J0 + 128).
  uint32_t rel[8];  // bit b of rel[a]: pair (8ty + a, tx + 16b) related
  bool any = false;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int64_t i = I0 + ty * 8 + a;
    uint32_t r = 0;
    if (i < n) {
      const uint4 x = *(const uint4*)(ta.S32 + i * ta.ld32 + (J0 >> 5));
      const uint32_t xw[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int c = tx + 16 * b;
        const int64_t j = J0 + c;
        if (((xw[c >> 5] >> (c & 31)) & 1u) && i < j) r |= 1u << b;
      }
    }
    rel[a] = r;
    any |= (r != 0);
  }
  const bool wave_any = __any(any);
  if (!__syncthreads_or(any)) return false;

  uint32_t acc[8][8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[a][b] = 0;

  const int64_t kbeg = I0;
  const int64_t kend = (J0 + BM < n ? J0 + BM : n);
  const int64_t nst = ceil_div(kend - kbeg, kStageBits);
  const int64_t row_bits = ta.ld32 * 32;
  Stage<BM> sa, sb;
  sa.init(ta.S32, ta.ld32, I0, n, kbeg);
  sb.init(ta.S32, ta.ld32, J0, n, kbeg);
  sa.fetch(0, kbeg, row_bits, I0, kbeg < I0 + BM, true);
  sb.fetch(0, kbeg, row_bits, J0, kbeg + kStageBits > J0, false);
  for (int64_t s = 0; s < nst; ++s) {
    __syncthreads();
    sa.store(As);
    sb.store(Bs);
    __syncthreads();
    if (s + 1 < nst) {
      const int64_t kb = kbeg + (s + 1) * kStageBits;
      sa.fetch(s + 1, kb, row_bits, I0, kb < I0 + BM, true);
      sb.fetch(s + 1, kb, row_bits, J0, kb + kStageBits > J0, false);
    }
    if (!wave_any) continue;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint4 aw[8], bw[8];
#pragma unroll
      for (int a = 0; a < 8; ++a) aw[a] = *(const uint4*)(As + lds_pos(ty * 8 + a, h));
#pragma unroll
      for (int b = 0; b < 8; ++b) bw[b] = *(const uint4*)(Bs + lds_pos(tx + 16 * b, h));
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          acc[a][b] += __popc(aw[a].x & bw[b].x);
          acc[a][b] += __popc(aw[a].y & bw[b].y);
          acc[a][b] += __popc(aw[a].z & bw[b].z);
          acc[a][b] += __popc(aw[a].w & bw[b].w);
        }
    }
  }
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b)
      if ((rel[a] >> b) & 1u) bin_add(lds_hist, ta.hist, acc[a][b], nbins, tmax);
  return true;
}

// ===========================================================================
// Single-instance kernels: persistent over the T(T+1)/2 tiles, longest first.
// ===========================================================================
template <int BM>
struct TileLds {
  uint32_t As[BM * kStageWords] __attribute__((aligned(16)));
  uint32_t Bs[BM * kStageWords] __attribute__((aligned(16)));
  uint32_t hist[kLdsBins];
  uint32_t maxbin;
  int slot;
};

template <int WM>
__global__ __launch_bounds__(kThreads, 1) void k_count_mfma(const uint64_t* __restrict__ S,
                                                            int64_t n, int64_t ld,
                                                            unsigned long long* __restrict__ hist,
                                                            unsigned int* __restrict__ counter) {
  constexpr int BM = 2 * WM * 32;
  __shared__ TileLds<BM> L;
  const int64_t T = ceil_div(n, BM);
  const int64_t ntiles = T * (T + 1) / 2;
  for (int b = threadIdx.x; b < kLdsBins; b += kThreads) L.hist[b] = 0;
  uint32_t tmax = 0;
  int64_t pairs_in_lds = 0;
  TileArgs ta{(const uint32_t*)S, 2 * ld, n, 0, 0, hist};
  for (;;) {
    const int64_t t = next_tile(counter, &L.slot);
    if (t >= ntiles) break;
    int64_t I, J;
    tile_of(t, T, &I, &J);
    if (pairs_in_lds > (1ll << 31) - (int64_t)BM * BM) {  // keep uint32 LDS bins exact
      flush_hist(L.hist, hist, n - 1, tmax, &L.maxbin);
      pairs_in_lds = 0;
    }
    ta.I0 = I * BM;
    ta.J0 = J * BM;
    if (mfma_tile<WM>(ta, L.As, L.Bs, L.hist, tmax)) pairs_in_lds += (int64_t)BM * BM;
  }
  flush_hist(L.hist, hist, n - 1, tmax, &L.maxbin);
}

__global__ __launch_bounds__(kThreads, 2) void k_count_bitset(const uint64_t* __restrict__ S,
                                                              int64_t n, int64_t ld,
                                                              unsigned long long* __restrict__ hist,
                                                              unsigned int* __restrict__ counter) {
  constexpr int BM = kBitsetTile;
  __shared__ TileLds<BM> L;
  const int64_t T = ceil_div(n, BM);
  const int64_t ntiles = T * (T + 1) / 2;
  for (int b = threadIdx.x; b < kLdsBins; b += kThreads) L.hist[b] = 0;
  uint32_t tmax = 0;
  int64_t pairs_in_lds = 0;
  TileArgs ta{(const uint32_t*)S, 2 * ld, n, 0, 0, hist};
  for (;;) {
    const int64_t t = next_tile(counter, &L.slot);
    if (t >= ntiles) break;
    int64_t I, J;
    tile_of(t, T, &I, &J);
    if (pairs_in_lds > (1ll << 31) - (int64_t)BM * BM) {
      flush_hist(L.hist, hist, n - 1, tmax, &L.maxbin);
      pairs_in_lds = 0;
    }
    ta.I0 = I * BM;
    ta.J0 = J * BM;
    if (bitset_tile(ta, L.As, L.Bs, L.hist, tmax)) pairs_in_lds += (int64_t)BM * BM;
  }
  flush_hist(L.hist, hist, n - 1, tmax, &L.maxbin);
}

// ===========================================================================
// Ensemble kernels: persistent over packed work items (instance << 16 | I << 8 | J),
// ordered longest first across all instances.  The LDS histogram belongs to one
// instance at a time and is flushed when the workgroup moves to another instance.
// Instance sizes are at most 8192, so every bin fits in LDS.
// ===========================================================================
template <int MODE>  // 0: bitset (128 tiles), 2 / 4: MFMA with WM = MODE
__global__ __launch_bounds__(kThreads, 1) void k_count_batch(const uint64_t* __restrict__ bits,
                                                             const BatchInst* __restrict__ inst,
                                                             const uint32_t* __restrict__ items,
                                                             int64_t nitems,
                                                             unsigned long long* __restrict__ hist,
                                                             unsigned int* __restrict__ counter) {
  constexpr int BM = MODE == 0 ? kBitsetTile : 2 * MODE * 32;
  __shared__ TileLds<BM> L;
  for (int b = threadIdx.x; b < kLdsBins; b += kThreads) L.hist[b] = 0;
  uint32_t tmax = 0;
  int cur = -1;
  TileArgs ta{nullptr, 0, 0, 0, 0, nullptr};
  for (;;) {
    const int64_t t = next_tile(counter, &L.slot);
    if (t >= nitems) break;
    const uint32_t it = items[t];
    const int k = (int)(it >> 16);
    if (k != cur) {
      if (cur >= 0) flush_hist(L.hist, ta.hist, ta.n - 1, tmax, &L.maxbin);
      cur = k;
      const BatchInst d = inst[k];
      ta.S32 = (const uint32_t*)(bits + d.bits_off);
      ta.ld32 = 2 * d.ld;
      ta.n = d.n;
      ta.hist = hist + d.hist_off;
    }
    ta.I0 = (int64_t)((it >> 8) & 255u) * BM;
    ta.J0 = (int64_t)(it & 255u) * BM;
    if (MODE == 0)
      bitset_tile(ta, L.As, L.Bs, L.hist, tmax);
    else
      mfma_tile<(MODE == 0 ? 2 : MODE)>(ta, L.As, L.Bs, L.hist, tmax);
  }
  if (cur >= 0) flush_hist(L.hist, ta.hist, ta.n - 1, tmax, &L.maxbin);
}

__global__ void k_fill_u64(uint64_t* __restrict__ p, int64_t count, uint64_t value) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

}  // namespace

int device_cu_count() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      cus = prop.multiProcessorCount;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

cs_status launch_fill_u64(uint64_t* p, int64_t count, uint64_t value, hipStream_t st) {
  if (count <= 0) return CS_OK;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, st, p, count,
                     value);
  CS_LAUNCH_CHECK();
  return CS_OK;
}

size_t histogram_ws_bytes(int64_t, int) { return 256; }

cs_status launch_histogram(const uint64_t* bits, int64_t n, int64_t ld, int counter, uint64_t* hist,
                           void* ws, hipStream_t st) {
  unsigned int* ctr = (unsigned int*)ws;
  cs_status s = launch_fill_u64(hist, n - 1, 0, st);
  if (s != CS_OK) return s;
  s = launch_fill_u64((uint64_t*)ws, 1, 0, st);
  if (s != CS_OK) return s;
  const int cus = device_cu_count();
  if (counter == CS_COUNT_MFMA) {
    if (n <= 4096) {
      const int64_t T = ceil_div(n, 128);
      unsigned grid = (unsigned)std::min<int64_t>(T * (T + 1) / 2, cus);
      hipLaunchKernelGGL(k_count_mfma<2>, dim3(grid), dim3(kThreads), 0, st, bits, n, ld,
                         (unsigned long long*)hist, ctr);
    } else {
      const int64_t T = ceil_div(n, 256);
      unsigned grid = (unsigned)std::min<int64_t>(T * (T + 1) / 2, cus);
      hipLaunchKernelGGL(k_count_mfma<4>, dim3(grid), dim3(kThreads), 0, st, bits, n, ld,
                         (unsigned long long*)hist, ctr);
    }
  } else {
    const int64_t T = ceil_div(n, 128);
    unsigned grid = (unsigned)std::min<int64_t>(T * (T + 1) / 2, 2 * cus);
    hipLaunchKernelGGL(k_count_bitset, dim3(grid), dim3(kThreads), 0, st, bits, n, ld,
                       (unsigned long long*)hist, ctr);
  }
  CS_LAUNCH_CHECK();
  return CS_OK;
}

cs_status launch_count_batch(int mode, const uint64_t* bits, const BatchInst* inst,
                             const uint32_t* items, int64_t nitems, uint64_t* hist,
                             unsigned int* counter, hipStream_t st) {
  if (nitems <= 0) return CS_OK;
  const int cus = device_cu_count();
  const int per_cu = mode == 4 ? 1 : 2;  // LDS: 80 KiB (256 tiles) or 72 KiB (128 tiles)
  unsigned grid = (unsigned)std::min<int64_t>(nitems, (int64_t)cus * per_cu);
  unsigned long long* h = (unsigned long long*)hist;
  switch (mode) {
    case 0:
      hipLaunchKernelGGL(k_count_batch<0>, dim3(grid), dim3(kThreads), 0, st, bits, inst, items,
                         nitems, h, counter);
      break;
    case 2:
      hipLaunchKernelGGL(k_count_batch<2>, dim3(grid), dim3(kThreads), 0, st, bits, inst, items,
                         nitems, h, counter);
      break;
    case 4:
      hipLaunchKernelGGL(k_count_batch<4>, dim3(grid), dim3(kThreads), 0, st, bits, inst, items,
                         nitems, h, counter);
      break;
    default: return CS_ERR_UNSUPPORTED;
  }
  CS_LAUNCH_CHECK();
  return CS_OK;
}

}  // namespace cs
