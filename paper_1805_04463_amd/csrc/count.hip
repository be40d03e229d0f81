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
//   - K staged through LDS 256 bits at a time; the triangular masks (k > i for A,
//     k < j for B) only matter on stages that overlap the tile's own diagonal
//     blocks and are applied only there;
//   - an epilogue that tests the related bit S[j][i] of each output and bins the
//     count into a per-workgroup LDS histogram (HB uint32 bins) or, beyond it,
//     straight into the global uint64 histogram; LDS bins are flushed at exit.
// The MFMA counter fills a 4-deep LDS ring with direct global->LDS DMA loads
// (buffer_load_dwordx4 ... lds; rows past n read as zero through the buffer
// descriptor's range), so three stages are in flight while one is multiplied and
// each stage costs one barrier.  The bitset counter prefetches one stage through
// registers.
// They differ in the inner product:
//   MFMA   bits are expanded to int8 0/1 in registers and multiplied on
//          v_mfma_i32_32x32x32_i8 with int32 accumulation (exact: counts < 2^31).
//          Because both operands are rows of S, any permutation of k inside a
//          32-bit word works if applied to A and B alike; the expansion used,
//          byte b of register q = bit (4h + q + 8b) of the word (h = lane >> 5),
//          costs two VALU ops per four bytes.
//   BITSET AND + v_bcnt_u32_b32 on 32-bit words, each thread an 8x8 block of pairs.
#include <type_traits>
#include <utility>

#include "common.h"

namespace cs {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;
constexpr int kStageBits = 256;         // K bits per LDS stage
constexpr int kStageWords = kStageBits / 32;
constexpr int kHalfRows = 129;  // half-major B stage of related-pair tiles: 128 rows + a zero row
constexpr int kBinsSingle = 12288;      // LDS histogram bins, single instance (48 KiB)
constexpr int kBinsBatch = 8192;        // LDS histogram bins, ensembles (n <= 8192)

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

// The same masks from the offset d = kw - g, for |d| < 2^30: the shift count is
// clamped to [0, 32] and the 64-bit shift gives the empty mask at 32.
__device__ inline uint32_t mask_above_d(int32_t d) {  // bits b with d + b > 0
  const int32_t s = min(max(1 - d, 0), 32);
  return (uint32_t)(0xFFFFFFFFull << s);
}
__device__ inline uint32_t mask_below_d(int32_t d) {  // bits b with d + b < 0
  const int32_t s = min(max(-d, 0), 32);
  return ~(uint32_t)(0xFFFFFFFFull << s);
}
// A tile-relative offset as int32: outside +-2^24 every mask is all-or-nothing anyway.
__device__ inline int32_t clamp_offset(int64_t v) {
  return (int32_t)(v < -(1 << 24) ? -(1 << 24) : (v > (1 << 24) ? (1 << 24) : v));
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
  // LAYOUT 0: the XOR-swizzled layout of lds_pos (dense tiles).  1: row r at
  // r * kStageWords, its halves at +0 and +4 words (A side of related-pair tiles, whose
  // reads take the second half through the instruction's immediate offset).  2: half-major,
  // half h of row r at (h * kHalfRows + r) * 4 words (B side of related-pair tiles: lanes
  // reading the same half of rows a few apart then fall in different bank groups).
  template <int LAYOUT = 0>
  __device__ inline void store(uint32_t* lds) const {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int c = threadIdx.x + q * kThreads;
      const int r = c >> 1, h = c & 1;
      const int pos = LAYOUT == 0 ? lds_pos(r, h)
                      : LAYOUT == 1 ? r * kStageWords + h * 4 : (h * kHalfRows + r) * 4;
      *(uint4*)(lds + pos) = v[q];
    }
  }
};

// Counts are at most n-2 by construction; the bound check keeps a histogram write in
// range whatever the inputs.  `tmax` tracks the largest LDS bin this thread touched.
template <int HB>
__device__ inline void bin_add(uint32_t* lds_hist, unsigned long long* hist, uint32_t bin,
                               int64_t nbins, uint32_t& tmax) {
  if (bin < (uint32_t)HB) {
    atomicAdd(lds_hist + bin, 1u);
    tmax = bin > tmax ? bin : tmax;
  } else if ((int64_t)bin < nbins) {
    atomicAdd(hist + bin, 1ull);
  }
}

// Adds the LDS bins [0, max touched] to the global histogram and clears them.
template <int HB>
__device__ inline void flush_hist(uint32_t* lds_hist, unsigned long long* hist, int64_t nbins,
                                  uint32_t& tmax, uint32_t* s_max) {
  __syncthreads();
  if (threadIdx.x == 0) *s_max = 0;
  __syncthreads();
  atomicMax(s_max, tmax);
  __syncthreads();
  int64_t lim = (int64_t)*s_max + 1;
  lim = lim < nbins ? lim : nbins;
  lim = lim < HB ? lim : HB;
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

// Arguments of the d'Alembertian epilogue: out[j] accumulates sum_m c_m sum_{L_m(j)} phi(i).
struct FieldArgs {
  const double* phi;
  double* out;
  double c0, c1, c2, c3;      // c_m for pairs with m interior elements (0 past the last layer)
};

struct TileArgs {
  const uint32_t* S32;        // instance matrix, as 32-bit words
  int64_t ld32;               // row stride in 32-bit words
  int64_t n;                  // points of the instance
  int64_t I0, J0;             // first row / first column of the output tile
  unsigned long long* hist;   // instance histogram (n-1 bins)
  FieldArgs f;                // d'Alembertian epilogue only
};

// ===========================================================================
// MFMA tile.  Workgroup tile BM x BM, four waves in 2x2, each WM x WM blocks of
// 32x32 outputs (WM = 4: 256x256 tile, 128x128 per wave, 256 int32 accumulators).
// Returns false (having done nothing) when no pair of the tile is related.
// ===========================================================================

// s_waitcnt with vmcnt = N and no wait on the other counters (gfx9 encoding).
template <int N>
__device__ inline void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// MFMA stages: 512 bits of K = 64 contiguous bytes of every panel row, so each DMA
// request covers half a 128-byte line and a line is consumed by two neighbouring
// stages.  Within a stage, row r's four 16-byte chunks sit at positions c ^ (r/4 mod 4)
// so that sixteen consecutive rows reading the same chunk hit distinct banks.
#ifndef CS_DMA_STEPS
#define CS_DMA_STEPS(steps) ((steps) / 2)
#endif
constexpr int kMStageBits = 512;
constexpr int kMStageU32 = kMStageBits / 32;  // uint32 words per row per stage
// Stages in the LDS ring: three for 256-row panels (one workgroup per CU), two for
// 128-row panels so that two workgroups fit in a CU's LDS.
template <int BM>
struct MRing {
  static constexpr int value = BM == 256 ? 3 : 2;
};

__device__ inline int mpos(int r, int c) { return r * kMStageU32 + ((c ^ ((r >> 2) & 3)) << 2); }

// One 16-byte-per-lane DMA request of a stage: load q (of BM*4/256) of a BM-row panel
// into an LDS stage buffer; request q of wave w writes slots q*256 + 64w + lane, slot
// s = 4r + (c ^ (r/4 mod 4)).
template <int BM>
__device__ inline void dma_one(__amdgpu_buffer_rsrc_t rsrc, uint32_t lds_stage_addr, int32_t voff,
                               int32_t kbyte, int q) {
  const uint32_t wave_off = __builtin_amdgcn_readfirstlane((threadIdx.x >> 6) * 64 * 16);
  // Rows past the panel's valid rows start beyond the descriptor's range, and stages past
  // the last carry a kbyte of 1 GiB (panels are below 1 GiB): either way the request reads
  // nothing.  Row part and kbyte are each below 2^30, so their sum does not wrap.
  const uint32_t vo = (uint32_t)voff + (uint32_t)kbyte;
  const uint32_t lds_addr = lds_stage_addr + wave_off + q * kThreads * 16;
  // Issued as inline assembly so the compiler does not add its own wait for the DMA
  // before every LDS read; completion is tracked explicitly with wait_vmcnt.  M0 holds
  // the DMA's LDS address and is declared clobbered (the compiler keeps nothing there
  // across the load); an LDS DMA needs one wait state after an SALU write of M0.
  asm volatile(
      "s_mov_b32 m0, %[la]\n\ts_nop 0\n\t"
      "buffer_load_dwordx4 %[vo], %[rs], 0 offen lds"
      :
      : [la] "s"(lds_addr), [vo] "v"(vo), [rs] "s"(rsrc)
      : "memory", "m0");
}

// Buffer descriptor of a panel (base, byte range), its fields made wave-uniform so they
// live in scalar registers whatever the compiler can prove about their origin.
__device__ inline __amdgpu_buffer_rsrc_t uniform_rsrc(const uint32_t* base, uint32_t bytes) {
  const uint64_t p = (uint64_t)(uintptr_t)base;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)p);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(p >> 32));
  const uint32_t nr = __builtin_amdgcn_readfirstlane(bytes);
  return __builtin_amdgcn_make_buffer_rsrc((void*)(uintptr_t)(((uint64_t)hi << 32) | lo), (short)0,
                                           (int)nr, 0x00020000);
}

// Panel byte offset of this thread's slot in DMA request 0 of a stage: slot s = tid holds
// row s/4, 16-byte chunk (s & 3) ^ (row/4 & 3); request q adds 64 rows, which leaves the
// chunk unchanged, so one register serves every request of both panels (same row stride).
// Rows past the panel's valid rows lie beyond its descriptor's range (valid rows * ld * 8
// bytes) and read as zero.
__device__ inline uint32_t dma_base(int64_t ld) {
  const uint32_t tid = threadIdx.x;
  return (tid >> 2) * (uint32_t)(ld * 8) + (((tid & 3u) ^ ((tid >> 4) & 3u)) << 4);
}

__device__ inline v4i unpack_i8(uint32_t x, uint32_t sh) {
  return (v4i){(int)((x >> sh) & 0x01010101u), (int)((x >> (sh + 1)) & 0x01010101u),
               (int)((x >> (sh + 2)) & 0x01010101u), (int)((x >> (sh + 3)) & 0x01010101u)};
}

__device__ inline uint32_t word_of(const uint4& v, int w) {
  return w == 0 ? v.x : w == 1 ? v.y : w == 2 ? v.z : v.w;
}

// fp4 matrix cores (v_mfma_scale_f32_32x32x64_f8f6f4, both operands e2m1).  A lane's
// 128-bit chunk (words q = 0..3) feeds four MFMAs, one per bit class c: register q of
// class c holds bits c, c+4, ..., c+28 of word q, each left in its own nibble, so no
// bit moves except for class 3.  Bit positions 0, 1, 2 of a nibble are the e2m1 codes
// 0.5, 1.0 and 2.0; the per-block E8M0 scales 2, 1, 1/2 (codes 128, 127, 126) bring
// every operand to 0 or 1, and class 3 is shifted down to position 0.  Products are
// 0 or 1 and every count is below 2^24, so the f32 accumulation is exact.
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

template <int C>
__device__ inline v8i unpack_fp4_class(const uint4& v) {
  if constexpr (C == 3)
    return (v8i){(int)((v.x >> 3) & 0x11111111u), (int)((v.y >> 3) & 0x11111111u),
                 (int)((v.z >> 3) & 0x11111111u), (int)((v.w >> 3) & 0x11111111u), 0, 0, 0, 0};
  constexpr uint32_t m = 0x11111111u << C;
  return (v8i){(int)(v.x & m), (int)(v.y & m), (int)(v.z & m), (int)(v.w & m), 0, 0, 0, 0};
}
template <int C>
constexpr int fp4_class_scale() { return C == 1 ? 127 : C == 2 ? 126 : 128; }

// Triangular masks applied in place to a stage in LDS, on the stages that overlap a
// diagonal block of the tile: A rows (i = I0 + r) keep k > i, B rows (j = J0 + r) keep
// k < j, for the stage's bits k in [kb, kb + 512).  The masks depend only on the row and
// k, so one pass serves every wave that reads the row.
// A side only when the stage starts at or before the last A row, B side only when it
// ends past the first B row; rows are dealt so that each wave takes one side.
template <int BM>
__device__ inline void mask_stage(uint32_t* As, uint32_t* Bs, int64_t kb, int64_t I0, int64_t J0) {
  static_assert(BM % 64 == 0, "a wave's rows lie on one side");
  const bool need_a = kb <= I0 + BM - 1, need_b = kb + kMStageBits > J0;
  const int32_t da = clamp_offset(kb - I0), db = clamp_offset(kb - J0);
  for (int x = threadIdx.x; x < 2 * BM; x += kThreads) {
    const bool is_a = __builtin_amdgcn_readfirstlane(x) < BM;  // the same for the whole wave
    if (!(is_a ? need_a : need_b)) continue;
    const int r = is_a ? x : x - BM;
    uint32_t* P = is_a ? As : Bs;
    const int32_t d0 = (is_a ? da : db) - r;  // first bit of the stage minus the row index
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      uint4 v = *(uint4*)(P + mpos(r, c));
      uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int32_t d = d0 + 128 * c + 32 * q;  // word start minus the row index
        w[q] &= is_a ? mask_above_d(d) : mask_below_d(d);
      }
      *(uint4*)(P + mpos(r, c)) = make_uint4(w[0], w[1], w[2], w[3]);
    }
  }
}

// f(std::integral_constant<int, i>) for i = 0 .. N-1, unrolled at compile time.
template <typename F, int... I>
__device__ inline void static_for_seq(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ inline void static_for(F&& f) {
  static_for_seq(f, std::make_integer_sequence<int, N>{});
}
// f(std::integral_constant<int, i>) for i = A .. B-1.
template <int A, typename F, int... I>
__device__ inline void static_for_from(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, A + I>{}), ...);
}
template <int A, int B, typename F>
__device__ inline void static_for_range(F&& f) {
  static_for_from<A>(f, std::make_integer_sequence<int, B - A>{});
}

// Chunk (of four per stage row) that half-wave hsel multiplies in half cc of a stage.
template <int WM>
__device__ inline int mchunk(int hsel, int cc) { return WM == 2 ? hsel + 2 * cc : 2 * hsel + cc; }

// One stage (512 bits of K = 4 chunks of 128) as a flat, software-pipelined sequence of
// k-steps.  Each half-wave multiplies two chunks of every row, its first in the stage's
// first half of k-steps and its second in the second half: with 256-row tiles lanes 0-31
// take chunks 0 and 1 and lanes 32-63 chunks 2 and 3; with 128-row tiles lanes 0-31 take
// chunks 0 and 2 and lanes 32-63 chunks 1 and 3, so the first half covers bits 0-255 of
// the stage and a last stage whose K range ends by bit 256 (`half`) skips the second half,
// whose B operands are masked to zero.  The MFMA's K order only has to be the same for A
// and B, and with either assignment each half-wave reads just the chunks it multiplies.  A chunk gives 4 fp4 k-steps
// (one per bit class) or 8 int8 k-steps (word w, nibble e of every byte: bits
// 32w + 4e + q + 8b in byte b of register q).  The operands of step t+1 are unpacked
// while the MFMAs of step t issue, and the scheduler is told to interleave them (one
// MFMA, then a share of the VALU work).
//
// Stages are chained without a gap.  On entry the registers hold this stage's chunk 0
// (aw[0], bw[0]) and the operands of its first step (af[0], bf[0]).  Chunk 1 is read
// at the first step.  After the first half every operand of the stage is in registers,
// so `mid` (wait for the next stage's DMA, barrier) both publishes the next stage and
// frees this stage's slot: the second half reads the next stage's chunk 0, issues the
// DMA pieces (`dma`) that refill this slot, and unpacks the next stage's first step.
// MODE 0: a plain stage follows; 1: the tile's last stage follows (`mid` masks it);
// 2: this is the tile's last stage.
template <int WM, bool FP4, int kLoads, int MODE, typename Acc, typename Frag, typename Mid,
          typename Dma, typename Fix>
__device__ inline void mfma_stage(Acc (&acc)[WM][WM], uint4 (&aw)[2][WM], uint4 (&bw)[2][WM],
                                  Frag (&af)[2][WM], Frag (&bf)[2][WM], const uint32_t* As,
                                  const uint32_t* Bs, const uint32_t* An, const uint32_t* Bn,
                                  int arow, int brow, int hsel, bool half, Mid&& mid,
                                  Dma&& dma, Fix&& fix) {
  constexpr int kSteps = FP4 ? 4 : 8;  // MFMA k-steps per 128-bit chunk
  constexpr int kT = 2 * kSteps;       // k-steps per stage
  constexpr int kPerStep = (kLoads + kSteps - 1) / kSteps;  // DMA pieces per step, 2nd half
  auto load_chunk = [&](const uint32_t* A, const uint32_t* B, int cc, uint4 (&a)[WM],
                        uint4 (&b)[WM]) {
    const int c = mchunk<WM>(hsel, cc);
#pragma unroll
    for (int mb = 0; mb < WM; ++mb) a[mb] = *(const uint4*)(A + mpos(arow + mb * 32, c));
#pragma unroll
    for (int nb = 0; nb < WM; ++nb) b[nb] = *(const uint4*)(B + mpos(brow + nb * 32, c));
  };
  auto unpack_step = [&](auto step, int cc, Frag (&fa)[WM], Frag (&fb)[WM]) {
    constexpr int u = decltype(step)::value;  // step within the chunk
#pragma unroll
    for (int mb = 0; mb < WM; ++mb) {
      if constexpr (FP4) fa[mb] = unpack_fp4_class<u>(aw[cc][mb]);
      else fa[mb] = unpack_i8(word_of(aw[cc][mb], u >> 1), 4u * (u & 1));
    }
#pragma unroll
    for (int nb = 0; nb < WM; ++nb) {
      if constexpr (FP4) fb[nb] = unpack_fp4_class<u>(bw[cc][nb]);
      else fb[nb] = unpack_i8(word_of(bw[cc][nb], u >> 1), 4u * (u & 1));
    }
  };
  auto mfmas = [&](auto step, const Frag (&fa)[WM], const Frag (&fb)[WM]) {
    constexpr int u = decltype(step)::value;
#pragma unroll
    for (int mb = 0; mb < WM; ++mb)
#pragma unroll
      for (int nb = 0; nb < WM; ++nb) {
        if constexpr (FP4) {
          constexpr int sc = fp4_class_scale<u>();
          acc[mb][nb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
              fa[mb], fb[nb], acc[mb][nb], 4, 4, 0, sc, 0, sc);
        } else {
          acc[mb][nb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[mb], fb[nb], acc[mb][nb], 0, 0, 0);
        }
      }
  };
  auto step = [&](auto tc) {
    constexpr int t = decltype(tc)::value;
    constexpr int cur = t & 1;
    if constexpr (t == 0) {
      load_chunk(As, Bs, 1, aw[1], bw[1]);
      fix(std::integral_constant<int, 0>{}, aw[1], bw[1]);
    }
    if constexpr (t == kSteps && MODE != 2) {
      load_chunk(An, Bn, 0, aw[0], bw[0]);
      fix(std::integral_constant<int, 1>{}, aw[0], bw[0]);
    }
    if constexpr (t >= kSteps) {
      // This step's share of the DMA (the stage is one basic block, so the per-step
      // scheduling barrier keeps it within the step).
      static_for<kPerStep>([&](auto qc) {
        constexpr int q = (t - kSteps) * kPerStep + decltype(qc)::value;
        if constexpr (q < kLoads) dma(std::integral_constant<int, q>{});
      });
    }
    constexpr bool unpack = t + 1 < kT || MODE != 2;
    constexpr int un = (t + 1) % kSteps, cn = ((t + 1) / kSteps) & 1;  // next stage: chunk 0
    if constexpr (unpack) unpack_step(std::integral_constant<int, un>{}, cn, af[cur ^ 1], bf[cur ^ 1]);
    mfmas(std::integral_constant<int, t % kSteps>{}, af[cur], bf[cur]);
    if constexpr (unpack) {
      // The next step's unpacking (2 WM fragments of 4 registers, 1 or 2 VALU ops each)
      // spread evenly between this step's WM*WM MFMAs.
      constexpr int kOps = FP4 ? (un == 3 ? 2 : 1) : 2;
      constexpr int kValu = kOps * 4 * 2 * WM / (WM * WM) + 1;
#pragma unroll
      for (int q = 0; q < WM * WM; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);      // one MFMA
        __builtin_amdgcn_sched_group_barrier(0x002, kValu, 0);  // then VALU
      }
    }
    // Keep each step's MFMAs in their own scheduling region: MFMAs of consecutive steps
    // update the same accumulators and must not be placed back to back.
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (t == kSteps - 1) mid();
  };
  static_for_range<0, kSteps>(step);
  if (MODE != 2 || !half) static_for_range<kSteps, kT>(step);
}

// Tiles of one ensemble row panel run one after another in a workgroup (J descending):
// the last stage of a 128-row tile fetches the next tile's first stage into the ring slot
// it leaves free, and the barrier at that stage's middle publishes it, so the next tile
// starts without a barrier or a wait.  rofs: the ring slot of the tile's stage 0; ready:
// that stage is in place; next_j0: the next tile's first column, or -1.
struct TileChain {
  int rofs = 0;
  bool ready = false;
  int64_t next_j0 = -1;
};

// EPI 0: histogram of the interval sizes of the related pairs.  EPI 1: d'Alembertian
// sums, per column j, of c_m phi(i) over the related pairs (i, j) with m interior elements.
// FITS: every count is below HB (instances of at most HB + 1 points), so the epilogue
// neither tracks the largest bin (the caller flushes all n - 1) nor needs its second pass.
template <int WM, int HB, bool FP4 = false, int EPI = 0, bool FITS = false>
__device__ __attribute__((always_inline)) inline bool mfma_tile(const TileArgs& ta, uint32_t* ring,
                                                                uint32_t* rel, uint32_t* lds_hist,
                                                                uint32_t& tmax, double* phis,
                                                                TileChain& chain) {
  using Acc = typename std::conditional<FP4, v16f, v16i>::type;
  constexpr int BM = 2 * WM * 32;
  constexpr int kStage = BM * kMStageU32;      // one panel stage, uint32 words
  constexpr int kPer = BM * 4 / kThreads;      // DMA loads per panel per thread
  constexpr int kLoads = 2 * kPer;             // per stage (A and B)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int hsel = lane >> 5, l32 = lane & 31;
  const int64_t n = ta.n, I0 = ta.I0, J0 = ta.J0, nbins = n - 1;

  const int64_t ld = ta.ld32 >> 1;
  const int64_t kbeg = I0;
  const int64_t kend = (J0 + BM < n ? J0 + BM : n);
  const int nst = (int)ceil_div(kend - kbeg, kMStageBits);
  const int64_t va = n - I0 < BM ? n - I0 : BM, vb = n - J0 < BM ? n - J0 : BM;
  const __amdgpu_buffer_rsrc_t ra =
      uniform_rsrc(ta.S32 + I0 * ta.ld32, (uint32_t)(va * ld * 8));
  const __amdgpu_buffer_rsrc_t rbf =
      uniform_rsrc(ta.S32 + J0 * ta.ld32, (uint32_t)(vb * ld * 8));
  const int32_t vbase = (int32_t)dma_base(ld);
  const int32_t rows64 = (int32_t)(64 * ld * 8);  // request stride: 64 panel rows, < 2^28
  const int32_t kbyte0 = (int32_t)(kbeg >> 3);

  // LDS byte address of the ring (the low 32 bits of a generic LDS pointer).
  const uint32_t ring_addr = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)ring);
  constexpr int R = MRing<BM>::value;
  constexpr bool kChain = WM == 2;  // 128-row tiles (two ring slots) chain their first stages
  const int rofs = kChain ? chain.rofs : 0;
  const bool ready = kChain && chain.ready;
  const bool fetch_next = kChain && chain.next_j0 >= 0;
  auto slot_of = [&](int st) { return (st + rofs) % R; };
  // DMA of stage st into its ring slot; past the last stage the requests are pushed out
  // of the descriptors' range (panels are below 1 GiB), so they read nothing.  Issuing
  // them anyway keeps the stage code free of branches, which would let the compiler
  // gather all requests in one place.
  auto dma_piece = [&](int st, auto qc) {
    constexpr int q = decltype(qc)::value;
    const uint32_t slot = ring_addr + slot_of(st) * 2 * kStage * 4;
    const int32_t kb = st < nst ? kbyte0 + st * (kMStageBits / 8) : (int32_t)0x40000000;
    constexpr int qp = q < kPer ? q : q - kPer;  // request within its panel
    if constexpr (q < kPer) dma_one<BM>(ra, slot, vbase, kb + qp * rows64, q);
    else dma_one<BM>(rbf, slot + kStage * 4, vbase, kb + qp * rows64, qp);
  };
  // The previous tile's global histogram atomics: retiring them here leaves the compiler
  // no outstanding memory operation to wait for inside the stage loop.
  wait_vmcnt<0>();
  for (int st = ready ? 1 : 0; st < R; ++st)  // prologue: stages 0 (unless in place) .. R-1
    static_for<kLoads>([&](auto qc) { dma_piece(st, qc); });
  // The B panel's K range starts at I0, so its first stage holds S[j][i] for every pair of
  // the tile: each lane takes the relation bits (i < j) of its pairs for the epilogue.
  // 128-row tiles keep them in registers (no LDS copy, and no tile skip: a tile without a
  // related pair is rare, and the skip costs a barrier); 256-row tiles, whose registers
  // are full, keep them in LDS and skip a tile without any.
  constexpr bool kRelRegs = WM == 2;
  uint32_t relw[WM][WM];
  uint32_t* const ring0 = ring + slot_of(0) * 2 * kStage;  // stage 0: A, then B
  if (!ready) {
    wait_vmcnt<(R - 1) * kLoads>();
    __syncthreads();
  }
  if constexpr (kRelRegs) {
    const uint32_t* Bs0 = ring0 + kStage;
    const int32_t dij = clamp_offset(I0 - J0);
#pragma unroll
    for (int nb = 0; nb < WM; ++nb)
#pragma unroll
      for (int mb = 0; mb < WM; ++mb) {
        const int br = wc * (WM * 32) + nb * 32 + l32, m = wr * WM + mb;
        relw[nb][mb] = Bs0[mpos(br, m >> 2) + (m & 3)] & mask_below_d(dij + 32 * m - br);
      }
  } else {
    bool any = false;
    const uint32_t* Bs0 = ring0 + kStage;
    const int32_t dij = clamp_offset(I0 - J0);
#pragma unroll
    for (int nb = 0; nb < WM; ++nb)
#pragma unroll
      for (int mb = 0; mb < WM; ++mb) {
        const int br = wc * (WM * 32) + nb * 32 + l32, m = wr * WM + mb;
        const uint32_t w = Bs0[mpos(br, m >> 2) + (m & 3)] & mask_below_d(dij + 32 * m - br);
        any |= w != 0u;
        if (hsel == 0) rel[((wave * WM + nb) * WM + mb) * 32 + l32] = w;
      }
    if (!__syncthreads_or(any)) {
      wait_vmcnt<0>();  // drain the DMA of later stages before the ring is reused
      return false;
    }
  }
  if constexpr (EPI == 1) {  // phi of the tile's rows, read by the epilogue
    for (int r = threadIdx.x; r < BM; r += kThreads) phis[r] = I0 + r < n ? ta.f.phi[I0 + r] : 0.0;
  }
  // Only the first and the last stage overlap a diagonal block (the A rows' block lies
  // in stage 0, the B rows' block in the last stage).  128-row tiles mask the operand
  // words in registers as they read them (no LDS pass and no barrier for it); 256-row
  // tiles, whose registers are full, mask both stages in LDS before they are read, the
  // first here, the last halfway through the stage before it.
  constexpr bool kRegMasks = WM == 2;
  if constexpr (!kRegMasks) {
    mask_stage<BM>(ring0, ring0 + kStage, kbeg, I0, J0);
    __syncthreads();
  }
  // Triangular masks on operand words in registers, as they are read: A rows
  // (i = I0 + row) keep k > i on stage 0, B rows (j = J0 + row) keep k < j on the last
  // stage; word q of this lane's chunk c of stage s holds k = kbeg + 512 s + 128 c + 32 q + b.
  auto mask_a = [&](uint4& v, int row, int64_t kw) {
    const int32_t d = clamp_offset(kw - (I0 + row));
    v.x &= mask_above_d(d);
    v.y &= mask_above_d(d + 32);
    v.z &= mask_above_d(d + 64);
    v.w &= mask_above_d(d + 96);
  };
  auto mask_b = [&](uint4& v, int row, int64_t kw) {
    const int32_t d = clamp_offset(kw - (J0 + row));
    v.x &= mask_below_d(d);
    v.y &= mask_below_d(d + 32);
    v.z &= mask_below_d(d + 64);
    v.w &= mask_below_d(d + 96);
  };

  using Frag = typename std::conditional<FP4, v8i, v4i>::type;
  const int arow = wr * WM * 32 + l32, brow = wc * WM * 32 + l32;
  uint4 aw[2][WM], bw[2][WM];
  Frag af[2][WM], bf[2][WM];
#pragma unroll
  for (int mb = 0; mb < WM; ++mb)
    aw[0][mb] = *(const uint4*)(ring0 + mpos(arow + mb * 32, mchunk<WM>(hsel, 0)));
#pragma unroll
  for (int nb = 0; nb < WM; ++nb)
    bw[0][nb] = *(const uint4*)(ring0 + kStage + mpos(brow + nb * 32, mchunk<WM>(hsel, 0)));
  if constexpr (kRegMasks) {
    const int64_t kw = kbeg + 128 * mchunk<WM>(hsel, 0);  // stage 0, this lane's first chunk
#pragma unroll
    for (int mb = 0; mb < WM; ++mb) mask_a(aw[0][mb], arow + mb * 32, kw);
    if (nst == 1)
#pragma unroll
      for (int nb = 0; nb < WM; ++nb) mask_b(bw[0][nb], brow + nb * 32, kw);
  }
#pragma unroll
  for (int mb = 0; mb < WM; ++mb) {
    if constexpr (FP4) af[0][mb] = unpack_fp4_class<0>(aw[0][mb]);
    else af[0][mb] = unpack_i8(aw[0][mb].x, 0u);
  }
#pragma unroll
  for (int nb = 0; nb < WM; ++nb) {
    if constexpr (FP4) bf[0][nb] = unpack_fp4_class<0>(bw[0][nb]);
    else bf[0][nb] = unpack_i8(bw[0][nb].x, 0u);
  }
  // fp4 histogram tiles start every accumulator at 2^23: the f32 sum 2^23 + count is then
  // exact (every addend is an integer and counts stay below 2^23) and its bit pattern is
  // 0x4B000000 + count, so the epilogue takes integer keys from the bits, without a
  // conversion.  The other tiles start at 0 and convert.
  constexpr bool kBias = FP4 && EPI == 0;
  constexpr uint32_t kB = kBias ? 0x4B000000u : 0u;
  Acc acc[WM][WM];
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WM; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        if constexpr (kBias) acc[a][b][e] = 8388608.0f;
        else acc[a][b][e] = 0;
      }
  auto key_of = [](auto v) -> uint32_t {  // kB + the count of an accumulator element
    if constexpr (kBias) return __builtin_bit_cast(uint32_t, v);
    else return (uint32_t)v;
  };

  auto stage = [&](auto modec, int s) {
    constexpr int MODE = decltype(modec)::value;
    const uint32_t* As = ring + slot_of(s) * 2 * kStage;
    const uint32_t* An = ring + slot_of(s + 1) * 2 * kStage;
    auto mid = [&]() {
      if constexpr (MODE != 2) wait_vmcnt<(R - 2) * kLoads>();  // stage s+1 has landed
      else if (fetch_next) wait_vmcnt<0>();  // the next tile's first stage has landed
      __syncthreads();
      if constexpr (MODE == 1 && !kRegMasks) {
        mask_stage<BM>(ring + slot_of(s + 1) * 2 * kStage, ring + slot_of(s + 1) * 2 * kStage + kStage,
                       kbeg + (int64_t)(s + 1) * kMStageBits, I0, J0);
        __syncthreads();
      }
    };
    // which 0: this stage's second chunk (A mask on stage 0, B mask on the last stage);
    // which 1: the next stage's first chunk (B mask when it is the last).
    auto fix = [&](auto whichc, uint4 (&a)[WM], uint4 (&b)[WM]) {
      constexpr int which = decltype(whichc)::value;
      if constexpr (!kRegMasks) return;
      const int64_t kw = kbeg + (int64_t)(s + which) * kMStageBits + 128 * mchunk<WM>(hsel, 1 - which);
      if constexpr (which == 0) {
        if (s == 0)
#pragma unroll
          for (int mb = 0; mb < WM; ++mb) mask_a(a[mb], arow + mb * 32, kw);
      }
      if constexpr ((which == 0 && MODE == 2) || (which == 1 && MODE == 1)) {
#pragma unroll
        for (int nb = 0; nb < WM; ++nb) mask_b(b[nb], brow + nb * 32, kw);
      }
    };
    auto dma = [&](auto qc) { dma_piece(s + R, qc); };  // refills this stage's slot
    // a last stage whose K range ends by its bit 256 skips its second half (128-row tiles)
    const bool half = WM == 2 && MODE == 2 && kend - (kbeg + (int64_t)s * kMStageBits) <= 256;
    if constexpr (MODE == 2 && kChain) {
      // The next tile's first stage (same A rows and K range, B rows from next_j0) into the
      // slot after this one, free since the previous stage's middle.
      if (fetch_next) {
        const __amdgpu_buffer_rsrc_t rbn =
            uniform_rsrc(ta.S32 + chain.next_j0 * ta.ld32, (uint32_t)(BM * ld * 8));
        const uint32_t slot = ring_addr + slot_of(s + 1) * 2 * kStage * 4;
        static_for<kLoads>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          constexpr int qp = q < kPer ? q : q - kPer;
          if constexpr (q < kPer) dma_one<BM>(ra, slot, vbase, kbyte0 + qp * rows64, q);
          else dma_one<BM>(rbn, slot + kStage * 4, vbase, kbyte0 + qp * rows64, qp);
        });
      }
    }
    mfma_stage<WM, FP4, kLoads, MODE>(acc, aw, bw, af, bf, As, As + kStage, An, An + kStage, arow,
                                      brow, hsel, half, mid, dma, fix);
  };
  int s = 0;
  for (; s + 2 < nst; ++s) stage(std::integral_constant<int, 0>{}, s);
  if (nst >= 2) stage(std::integral_constant<int, 1>{}, s++);
  stage(std::integral_constant<int, 2>{}, s);
  wait_vmcnt<0>();  // the out-of-range requests of the last stages, before the ring is reused
  if constexpr (kChain) {
    chain.rofs = slot_of(nst);  // the next tile's stage 0 went to the slot after the last
    chain.ready = fetch_next;
  }

  if constexpr (EPI == 0) {
  // Epilogue.  32x32 accumulator layout: lane holds column (lane & 31) and rows
  // 8*(e/4) + 4*(lane/32) + (e%4) for e = 0..15.  Branch-free binning: key = the pair's
  // count if it is related, else 0xFFFFFFFF (unrelated pairs all have count 0).  Every
  // element issues one LDS add, to min(key, HB + lane): its bin when key < HB, otherwise
  // a word past the bins (this lane's own one, or for HB <= key < HB + lane another
  // lane's), which is never flushed, so misses touch no bin.  tmax, the flush range,
  // follows the largest related key.  Counts of HB or more are rare: a second pass over
  // the block, behind a wave-uniform test, adds them to the global histogram.  Keys carry
  // the offset kB (fp4) until the LDS address is formed.
  const uint32_t spare = kB + (uint32_t)HB + (uint32_t)lane;
#pragma unroll
  for (int nb = 0; nb < WM; ++nb) {
#pragma unroll
    for (int mb = 0; mb < WM; ++mb) {
      const uint32_t w = (kRelRegs ? relw[nb][mb] : rel[((wave * WM + nb) * WM + mb) * 32 + l32]) >> (4 * hsel);
      if (!__ballot(w != 0u)) continue;  // no related pair in this 32x32 block
      const int32_t wn = (int32_t)~w;
      uint32_t big = 0;  // max over the block of key + 1 (0 for unrelated pairs)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int sh = (e >> 2) * 8 + (e & 3);
        // bit sh of wn, sign-extended: all ones for an unrelated pair, zero for a related one
        const uint32_t un = (uint32_t)__builtin_amdgcn_sbfe(wn, sh, 1);
        const uint32_t key = key_of(acc[mb][nb][e]) | un;
        const uint32_t slot = key < spare ? key : spare;
        atomicAdd(lds_hist + (slot - kB), 1u);
        if constexpr (!FITS) big = key + 1u > big ? key + 1u : big;
      }
      if constexpr (FITS) continue;
      if (big) tmax = big - 1u - kB > tmax ? big - 1u - kB : tmax;
      if (__ballot(big > kB + (uint32_t)HB)) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int sh = (e >> 2) * 8 + (e & 3);
          const uint32_t bin = key_of(acc[mb][nb][e]) - kB;
          if (((w >> sh) & 1u) && bin >= (uint32_t)HB && (int64_t)bin < nbins)
            atomicAdd(ta.hist + bin, 1ull);
        }
      }
    }
  }
  } else {
    // d'Alembertian epilogue: per column j of this lane, sum c_m phi(i) over the lane's
    // related rows i with m interior elements.  c_m comes from a table in LDS after the
    // rows' phi, indexed by min(key, 4): entry 4 is 0, for m >= 4 and for unrelated pairs
    // (key 0xFFFFFFFF).  Each row's phi is read once for the WM column blocks.  The two
    // half-waves hold the same columns and are combined by a lane exchange, and each wave
    // row adds its partial sums to out[j] with one fp64 atomic per column.
    const double* ctab = phis + BM;
    double part[WM];
#pragma unroll
    for (int nb = 0; nb < WM; ++nb) part[nb] = 0.0;
#pragma unroll
    for (int mb = 0; mb < WM; ++mb) {
      int32_t wn[WM];
      bool any = false;
#pragma unroll
      for (int nb = 0; nb < WM; ++nb) {
        const uint32_t w = (kRelRegs ? relw[nb][mb] : rel[((wave * WM + nb) * WM + mb) * 32 + l32]) >> (4 * hsel);
        any |= w != 0u;
        wn[nb] = (int32_t)~w;
      }
      if (!__ballot(any)) continue;  // no related pair in this row block
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int sh = (e >> 2) * 8 + (e & 3);
        const int r = wr * (WM * 32) + mb * 32 + (e >> 2) * 8 + hsel * 4 + (e & 3);
        const double ph = phis[r];
#pragma unroll
        for (int nb = 0; nb < WM; ++nb) {
          const uint32_t key =
              (uint32_t)acc[mb][nb][e] | (uint32_t)__builtin_amdgcn_sbfe(wn[nb], sh, 1);
          part[nb] = __fma_rn(ctab[key < 4u ? key : 4u], ph, part[nb]);
        }
      }
    }
#pragma unroll
    for (int nb = 0; nb < WM; ++nb) {
      const double sum = part[nb] + __shfl_xor(part[nb], 32);
      const int64_t j = J0 + wc * (WM * 32) + nb * 32 + l32;
      if (hsel == 0 && sum != 0.0 && j < n) atomicAdd(ta.f.out + j, sum);
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

template <int HB>
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
      if ((rel[a] >> b) & 1u) bin_add<HB>(lds_hist, ta.hist, acc[a][b], nbins, tmax);
  return true;
}

// ===========================================================================
// Related-pair tile (bitset counter, Alg. "Optimized Interval Abundance Measurement":
// only related pairs are counted).  Sprinkled orders are sparse near the diagonal and
// dense far from it: in a 3+1 diamond three quarters of the 128 x 128 tiles relate fewer
// than one pair in ten, while the tiles with half or more of their pairs related hold
// over half of the related-pair work.  So each tile first collects its related pairs and
// then takes one of two paths:
//   - few related pairs (at most `pair_max` tasks): the pairs are packed into tasks of
//     up to four related columns of one row; each thread holds up to kPairSlots tasks in
//     registers and, per staged K chunk, ANDs the task row's words with each of its
//     columns' words and accumulates v_bcnt.  One A read serves four columns.
//   - many related pairs: the dense 8 x 8 register-blocked product of bitset_tile.
// Tasks come from a workgroup scan of the rows' task counts (ceil(related / 4)); a
// task's columns are the row's related columns number 4k .. 4k+3 in its 128-bit slice.
// Unused columns of a task read a zero row kept after the B stage.
// ===========================================================================
constexpr int kPairGroup = 4;                        // related columns per task
constexpr int kPairSlots = 9;                        // tasks per thread
constexpr int kPairTaskMax = kPairSlots * kThreads;  // tasks per tile on the pair path
constexpr int kZeroRow = kBitsetTile;                // B-stage row that stays zero

// Exclusive prefix sum of v over the workgroup in thread order; *total gets the sum.
// wsum: kThreads / 64 words of LDS.
__device__ inline int block_exclusive_scan(int v, int* wsum, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    const int sw = wsum[w];
    off += w < wave ? sw : 0;
    tot += sw;
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

struct PairLds {
  uint32_t rowmask[kBitsetTile * 4];  // related columns of each tile row (j > i only)
  uint16_t task[kPairTaskMax];        // (row << 8) | number of the task's first column
  int wsum[kThreads / 64];
};

// Returns 0 when no pair of the tile is related (nothing done), 1 after the pair path,
// 2 when the tile has too many related pairs for it (nothing done: the caller takes the
// dense path).
template <int HB>
__device__ inline int pair_tile(const TileArgs& ta, uint32_t* As, uint32_t* Bs, PairLds& P,
                                uint32_t* lds_hist, uint32_t& tmax, int pair_max) {
  constexpr int BM = kBitsetTile;
  const int64_t n = ta.n, I0 = ta.I0, J0 = ta.J0, nbins = n - 1;
  const int tid = threadIdx.x, wave = tid >> 6;

  // Related columns: thread (r, h) = (tid / 2, tid % 2) takes the 64 columns
  // [J0 + 64h, J0 + 64h + 64) of row I0 + r; on a diagonal tile only j > i.
  int ntask;
  {
    const int r = tid >> 1, h = tid & 1;
    const int64_t i = I0 + r;
    uint64_t m = 0;
    if (i < n) m = *(const uint64_t*)(ta.S32 + i * ta.ld32 + (J0 >> 5) + 2 * h);
    if (I0 == J0) {
      const int lo = r + 1 - 64 * h;  // keep column bits b >= lo
      m = lo >= 64 ? 0ull : (lo <= 0 ? m : m & (~0ull << lo));
    }
    P.rowmask[4 * r + 2 * h] = (uint32_t)m;
    P.rowmask[4 * r + 2 * h + 1] = (uint32_t)(m >> 32);
    const int c = __popcll(m);
    const int row = c + __shfl_xor(c, 1);
    const int nt = h == 0 ? (row + kPairGroup - 1) / kPairGroup : 0;
    const int off = block_exclusive_scan(nt, P.wsum, &ntask);
    if (ntask == 0) return 0;
    if (ntask > pair_max) return 2;
    for (int k = 0; k < nt; ++k) P.task[off + k] = (uint16_t)((r << 8) | (kPairGroup * k));
    // the zero row of both halves of the B stage (the dense path shares the buffer)
    if (tid < 2 * 4) Bs[((tid >> 2) * kHalfRows + kZeroRow) * 4 + (tid & 3)] = 0u;
  }
  __syncthreads();

  // Tasks q * kThreads + tid -> byte offsets of the task row in the A stage and of its
  // columns' rows in the B stage (the zero row where a task has fewer columns).
  constexpr int kRowBytes = kStageWords * 4;      // A stage: row-major
  constexpr uint32_t kZeroOff = kZeroRow * 16;      // B stage: half-major, 16 bytes per row
  uint32_t aoff[kPairSlots], boff[kPairSlots][kPairGroup], acc[kPairSlots][kPairGroup];
#pragma unroll
  for (int q = 0; q < kPairSlots; ++q) {
    const int t = q * kThreads + tid;
    aoff[q] = 0;
#pragma unroll
    for (int g = 0; g < kPairGroup; ++g) {
      boff[q][g] = kZeroOff;
      acc[q][g] = 0;
    }
    if (t < ntask) {
      const uint32_t e = P.task[t];
      const int r = (int)(e >> 8);
      int skip = (int)(e & 255u);
      aoff[q] = (uint32_t)(r * kRowBytes);
      // Walk the row's 128-bit slice: skip `skip` related columns, take the next four.
      int w = 0;
      uint32_t x = P.rowmask[4 * r];
      while (w < 3 && skip >= __popc(x)) {
        skip -= __popc(x);
        x = P.rowmask[4 * r + (++w)];
      }
      for (; skip > 0; --skip) x &= x - 1u;
#pragma unroll
      for (int g = 0; g < kPairGroup; ++g) {
        while (x == 0u && w < 3) x = P.rowmask[4 * r + (++w)];
        if (x != 0u) {
          boff[q][g] = (uint32_t)((32 * w + __ffs(x) - 1) * 16);
          x &= x - 1u;
        }
      }
    }
  }

  const int64_t kbeg = I0;
  const int64_t kend = (J0 + BM < n ? J0 + BM : n);
  const int64_t nst = ceil_div(kend - kbeg, kStageBits);
  const int64_t row_bits = ta.ld32 * 32;
  // Two stages in flight through registers (the pair path has little arithmetic per stage
  // to hide a fetch behind): stage s + 2 is fetched into the buffer stage s just left.
  Stage<BM> sa[2], sb[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    sa[u].init(ta.S32, ta.ld32, I0, n, kbeg);
    sb[u].init(ta.S32, ta.ld32, J0, n, kbeg);
    if (u < nst) {
      const int64_t kb = kbeg + u * kStageBits;
      sa[u].fetch(u, kb, row_bits, I0, kb < I0 + BM, true);
      sb[u].fetch(u, kb, row_bits, J0, kb + kStageBits > J0, false);
    }
  }
  const char* Ab = (const char*)As;
  const char* Bb = (const char*)Bs;
  auto stage = [&](auto uc, int64_t s) {
    constexpr int u = decltype(uc)::value;
    __syncthreads();
    sa[u].template store<1>(As);
    sb[u].template store<2>(Bs);
    __syncthreads();
    if (s + 2 < nst) {
      const int64_t kb = kbeg + (s + 2) * kStageBits;
      sa[u].fetch(s + 2, kb, row_bits, I0, kb < I0 + BM, true);
      sb[u].fetch(s + 2, kb, row_bits, J0, kb + kStageBits > J0, false);
    }
#pragma unroll
    for (int q = 0; q < kPairSlots; ++q) {
      if (q * kThreads + wave * 64 < ntask) {  // wave-uniform: a task in this slot
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const uint4 a = *(const uint4*)(Ab + aoff[q] + 16 * h);
#pragma unroll
          for (int g = 0; g < kPairGroup; ++g) {
            const uint4 b = *(const uint4*)(Bb + boff[q][g] + 16 * kHalfRows * h);
            acc[q][g] += __popc(a.x & b.x);
            acc[q][g] += __popc(a.y & b.y);
            acc[q][g] += __popc(a.z & b.z);
            acc[q][g] += __popc(a.w & b.w);
          }
        }
      }
    }
  };
  int64_t s = 0;
  for (; s + 1 < nst; s += 2) {
    stage(std::integral_constant<int, 0>{}, s);
    stage(std::integral_constant<int, 1>{}, s + 1);
  }
  if (s < nst) stage(std::integral_constant<int, 0>{}, s);
#pragma unroll
  for (int q = 0; q < kPairSlots; ++q)
#pragma unroll
    for (int g = 0; g < kPairGroup; ++g)
      if (boff[q][g] != kZeroOff) bin_add<HB>(lds_hist, ta.hist, acc[q][g], nbins, tmax);
  return 1;
}

// ===========================================================================
// XCD-aware tile schedule for the MFMA counters.
//
// The MI355X's 256 CUs sit in 8 XCDs, each with its own L2.  Tiles that share a row
// panel of S (same I) or a column panel (same J) can share its fetches from HBM when
// they run at the same time on the same XCD.  So output tiles are grouped into
// rectangles of 4 x 8 tiles (I in [4a, 4a+4), J in [8b, 8b+8)): 32 tiles, one per CU of
// an XCD, reading 4 + 8 panels instead of 64.  Rectangles are ordered by their
// distance from the diagonal (k = 2b - a, cost ~ J - I), longest first, and dealt
// round-robin to 8 queues; a workgroup serves the queue of the XCD it runs on
// (hardware register XCC_ID) and then takes work from the other queues, so all tiles
// are done whatever the mapping of workgroups to XCDs.
// ===========================================================================
constexpr int kRA = 4, kRB = 8, kRect = kRA * kRB, kQueues = 8;
constexpr int64_t kRectMinTiles = 2 * kRect * kQueues;  // below: a single queue
constexpr int kMaxK = 2048;  // diagonals of the rectangle grid served by the queues (T <= 8184)

struct RectSched {
  int64_t T, NA, NB, R;     // tiles per side, rectangle grid, rectangles touching j >= i
  int K, kmax;              // k = kmax - index, index in [0, K)
};

__device__ inline bool rect_sched_fits(int64_t T) { return 2 * ceil_div(T, kRB) + 2 <= kMaxK; }

// First b of the k-diagonal: a = 2b - k >= 0 and b >= 0.
__device__ inline int64_t rect_first_b(int64_t k) { return k > 0 ? (k + 1) / 2 : 0; }

// sum_{m=0}^{x} floor(m / 2) for x >= -1, and 1 at x = -2, so that G(q) - G(p - 1) is the
// sum over m in [p, q] for every p >= -1.
__device__ inline int64_t floor_half_sum(int64_t x) {
  return x == -2 ? 1 : (x < 0 ? 0 : ((x + 1) / 2) * (x / 2));
}

// Rectangles on the diagonals k0 .. kmax.  The k-diagonal holds the b in
// [rect_first_b(k), min(NB - 1, floor((NA - 1 + k) / 2))]: NB - ceil(k/2) of them from
// kc = 2 NB - 1 - NA up, floor((NA - 1 + k) / 2) - ceil(k/2) + 1 below (never negative);
// both are sums of floor(m / 2) over ranges of m.
__device__ inline int64_t rect_prefix(const RectSched& rs, int64_t k0) {
  const int64_t kmax = rs.kmax;
  if (k0 > kmax) return 0;
  const int64_t kc = 2 * rs.NB - 1 - rs.NA;
  int64_t tot = 0;
  const int64_t a = k0 > kc ? k0 : kc;
  if (a <= kmax)  // sum ceil(k/2) over [a, kmax] = sum floor(m/2) over m in [a+1, kmax+1]
    tot += (kmax - a + 1) * rs.NB - (floor_half_sum(kmax + 1) - floor_half_sum(a));
  const int64_t b = kmax < kc - 1 ? kmax : kc - 1;
  if (k0 <= b) {
    const int64_t c = rs.NA - 1;
    tot += (floor_half_sum(b + c) - floor_half_sum(k0 + c - 1)) -
           (floor_half_sum(b + 1) - floor_half_sum(k0)) + (b - k0 + 1);
  }
  return tot;
}

// The schedule's sizes, from T alone: uniform values, so the lookups below run on the
// scalar unit.
__device__ inline RectSched rect_sched_make(int64_t T) {
  RectSched rs;
  rs.T = T;
  rs.NA = ceil_div(T, kRA);
  rs.NB = ceil_div(T, kRB);
  rs.kmax = (int)(2 * (rs.NB - 1));
  rs.K = rs.kmax + 2;  // k from kmax down to -1 (k >= -1 <=> rectangle reaches j >= i)
  rs.R = rect_prefix(rs, -1);
  return rs;
}

// Item q of queue x -> tile (I, J); false if the slot is past the queue or no tile.
__device__ inline bool rect_tile(const RectSched& rs, int x, int64_t q, int64_t* I, int64_t* J) {
  const int64_t r = (q / kRect) * kQueues + x;
  if (r >= rs.R) return false;
  int lo = 0, hi = rs.K - 1;  // last t whose diagonals above hold at most r rectangles
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (rect_prefix(rs, rs.kmax - mid + 1) <= r) lo = mid; else hi = mid - 1;
  }
  const int64_t k = rs.kmax - lo;
  const int64_t b = rect_first_b(k) + (r - rect_prefix(rs, k + 1));
  const int64_t a = 2 * b - k;
  const int p = (int)(q % kRect);
  *I = kRA * a + p / kRB;
  *J = kRB * b + p % kRB;
  return *I <= *J && *J < rs.T;
}

__device__ inline int64_t rect_queue_len(const RectSched& rs, int x) {
  return rs.R > x ? ((rs.R - x + kQueues - 1) / kQueues) * kRect : 0;
}

__device__ inline int xcc_id() {
  return (int)__builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11)) & (kQueues - 1);
}

// ===========================================================================
// Single-instance kernels: persistent over the T(T+1)/2 tiles, longest first.
// ===========================================================================
template <int BM, int HB>
struct MfmaLds {
  uint32_t ring[MRing<BM>::value * 2 * BM * kMStageU32] __attribute__((aligned(16)));
  uint32_t rel[BM == 128 ? 1 : BM * BM / 32];  // relation bits of the tile's pairs (i < j);
                                              // 128-row tiles keep theirs in registers
  double phis[BM + 8];         // phi of the tile's rows, then c_0 .. c_3, 0 (d'Alembertian)
  uint32_t hist[HB + 64];      // bins, then one spare word per lane (never flushed)
  uint32_t maxbin;
  int slot;
};
template <int HB>
struct BitsetLds {
  uint32_t As[kBitsetTile * kStageWords] __attribute__((aligned(16)));
  uint32_t Bs[2 * kHalfRows * 4] __attribute__((aligned(16)));  // dense, or half-major + zero row
  PairLds pairs;
  uint32_t hist[HB];
  uint32_t maxbin;
  int slot;
};

template <int WM, bool FP4, int EPI>
__global__ __launch_bounds__(kThreads, 1) void k_count_mfma(const uint64_t* __restrict__ S,
                                                            int64_t n, int64_t ld,
                                                            unsigned long long* __restrict__ hist,
                                                            unsigned int* __restrict__ counter,
                                                            FieldArgs f) {
  constexpr int BM = 2 * WM * 32, HB = kBinsSingle;
  __shared__ MfmaLds<BM, HB> L;  // 96 KiB ring + 48 KiB bins + 8 KiB relation bits at WM = 4
  const int64_t T = ceil_div(n, BM);
  if constexpr (EPI == 0)  // the bins a count can reach
    for (int b = threadIdx.x; b < HB && b < n - 1; b += kThreads) L.hist[b] = 0;
  if constexpr (EPI == 1)  // c_m table after the rows' phi (read after the first barrier)
    if (threadIdx.x < 5)
      L.phis[BM + threadIdx.x] = threadIdx.x == 0 ? f.c0 : threadIdx.x == 1 ? f.c1
                                 : threadIdx.x == 2 ? f.c2 : threadIdx.x == 3 ? f.c3 : 0.0;
  uint32_t tmax = 0;
  int64_t pairs_in_lds = 0;
  TileArgs ta{(const uint32_t*)S, 2 * ld, n, 0, 0, hist, f};
  // Rectangle queues per XCD while the table fits and there are enough tiles to share
  // panels (a workgroup that runs out of work probes every queue once, one global atomic
  // each, before it exits); otherwise one queue, longest K-range first.
  const bool rect = rect_sched_fits(T) && T * (T + 1) / 2 >= kRectMinTiles;
  const RectSched rs = rect_sched_make(rect ? T : 1);
  const int x0 = xcc_id();
  const int64_t ntiles = T * (T + 1) / 2;
  // Small matrices launch a workgroup per tile: each takes the tile of its own index,
  // without the queue's two atomic round trips.
  const bool direct = !rect && ntiles <= (int64_t)gridDim.x;
  bool taken = false;
  int probe = 0;
  for (;;) {
    int64_t I, J;
    if (rect) {
      if (probe >= kQueues) break;
      const int x = (x0 + probe) & (kQueues - 1);
      const int64_t q = __builtin_amdgcn_readfirstlane((int)next_tile(counter + x, &L.slot));
      if (q >= rect_queue_len(rs, x)) {
        ++probe;
        continue;
      }
      if (!rect_tile(rs, x, q, &I, &J)) continue;
    } else {
      int64_t t;
      if (direct) {
        if (taken) break;
        taken = true;
        t = blockIdx.x;
      } else {
        t = next_tile(counter, &L.slot);
        if (t >= ntiles) break;
      }
      tile_of(t, T, &I, &J);
    }
    if (EPI == 0 && pairs_in_lds > (1ll << 31) - (int64_t)BM * BM) {  // uint32 LDS bins exact
      flush_hist<HB>(L.hist, hist, n - 1, tmax, &L.maxbin);
      pairs_in_lds = 0;
    }
    ta.I0 = I * BM;
    ta.J0 = J * BM;
    TileChain none;
    if (mfma_tile<WM, HB, FP4, EPI>(ta, L.ring, L.rel, L.hist, tmax, L.phis, none))
      pairs_in_lds += (int64_t)BM * BM;
  }
  if constexpr (EPI == 0) flush_hist<HB>(L.hist, hist, n - 1, tmax, &L.maxbin);
}

__global__ __launch_bounds__(kThreads, 2) void k_count_bitset(const uint64_t* __restrict__ S,
                                                              int64_t n, int64_t ld,
                                                              unsigned long long* __restrict__ hist,
                                                              unsigned int* __restrict__ counter,
                                                              int pair_max) {
  constexpr int BM = kBitsetTile, HB = kBinsSingle;
  __shared__ BitsetLds<HB> L;
  const int64_t T = ceil_div(n, BM);
  const int64_t ntiles = T * (T + 1) / 2;
  // the bins a count can reach
  for (int b = threadIdx.x; b < HB && b < n - 1; b += kThreads) L.hist[b] = 0;
  uint32_t tmax = 0;
  int64_t pairs_in_lds = 0;
  TileArgs ta{(const uint32_t*)S, 2 * ld, n, 0, 0, hist};
  for (;;) {
    const int64_t t = next_tile(counter, &L.slot);
    if (t >= ntiles) break;
    int64_t I, J;
    tile_of(t, T, &I, &J);
    if (pairs_in_lds > (1ll << 31) - (int64_t)BM * BM) {
      flush_hist<HB>(L.hist, hist, n - 1, tmax, &L.maxbin);
      pairs_in_lds = 0;
    }
    ta.I0 = I * BM;
    ta.J0 = J * BM;
    const int path = pair_tile<HB>(ta, L.As, L.Bs, L.pairs, L.hist, tmax, pair_max);
    if (path == 2) bitset_tile<HB>(ta, L.As, L.Bs, L.hist, tmax);
    if (path) pairs_in_lds += (int64_t)BM * BM;
  }
  flush_hist<HB>(L.hist, hist, n - 1, tmax, &L.maxbin);
}

// ===========================================================================
// Ensemble kernels: persistent over packed row-panel items (instance << 16 | I << 8):
// one item is every tile (I, J >= I) of one instance's row panel I, longest first.
// The items sit in one queue per XCD, each queue whole instances one after another: a
// workgroup serves the queue of the XCD it runs on (hardware register XCC_ID), so the
// workgroups of an XCD work on the same matrix at once and share its panels in that
// XCD's L2, then takes work from the other queues.  The LDS histogram belongs to one
// instance at a time and is flushed when the workgroup moves to another instance.
// Instance sizes are at most 8192, so every bin fits in LDS.
// ===========================================================================
template <int MODE>  // 0: bitset (128 tiles), 2 / 4: MFMA with WM = MODE
struct BatchLdsOf {
  using type = MfmaLds<2 * MODE * 32, kBinsBatch>;
};
template <>
struct BatchLdsOf<0> {
  using type = BitsetLds<kBinsBatch>;
};

static_assert(kBinsBatch >= kBatchMaxN - 1, "ensemble counts fit the LDS bins");

template <int MODE, bool FP4 = false>
__global__ __launch_bounds__(kThreads, MODE == 4 ? 1 : 2) void k_count_batch(
    const uint64_t* __restrict__ bits, const BatchInst* __restrict__ inst,
    const uint32_t* __restrict__ items, BatchQueues queues, unsigned long long* __restrict__ hist,
    unsigned int* __restrict__ counter, int pair_max) {
  constexpr int BM = MODE == 0 ? kBitsetTile : 2 * MODE * 32, HB = kBinsBatch;
  __shared__ typename BatchLdsOf<MODE>::type L;
  for (int b = threadIdx.x; b < HB; b += kThreads) L.hist[b] = 0;
  uint32_t tmax = 0;
  int cur = -1;
  TileArgs ta{nullptr, 0, 0, 0, 0, nullptr};
  const int x0 = xcc_id();
  int probe = 0;
  for (;;) {
    if (probe >= kBatchQueues) break;
    const int x = (x0 + probe) & (kBatchQueues - 1);
    const int64_t q = next_tile(counter + x, &L.slot);
    if (q >= (int64_t)(queues.off[x + 1] - queues.off[x])) {
      ++probe;
      continue;
    }
    const uint32_t it = items[queues.off[x] + q];
    const int k = (int)(it >> 16);
    if (k != cur) {
      if (cur >= 0) flush_hist<HB>(L.hist, ta.hist, ta.n - 1, tmax, &L.maxbin);
      cur = k;
      const BatchInst d = inst[k];
      ta.S32 = (const uint32_t*)(bits + d.bits_off);
      ta.ld32 = 2 * d.ld;
      ta.n = d.n;
      ta.hist = hist + d.hist_off;
      if constexpr (MODE != 0) tmax = (uint32_t)(d.n - 2);  // FITS: flush every bin
    }
    const int64_t I = (int64_t)((it >> 8) & 255u);
    const int64_t T = ceil_div(ta.n, BM);
    ta.I0 = I * BM;
    TileChain chain;
    for (int64_t J = T - 1; J >= I; --J) {
      ta.J0 = J * BM;
      chain.next_j0 = J > I ? (J - 1) * BM : -1;
      if constexpr (MODE == 0) {
        if (pair_tile<HB>(ta, L.As, L.Bs, L.pairs, L.hist, tmax, pair_max) == 2)
          bitset_tile<HB>(ta, L.As, L.Bs, L.hist, tmax);
      } else
        mfma_tile<MODE, HB, FP4, 0, true>(ta, L.ring, L.rel, L.hist, tmax, nullptr, chain);
    }
  }
  if (cur >= 0) flush_hist<HB>(L.hist, ta.hist, ta.n - 1, tmax, &L.maxbin);
}

__global__ void k_fill_u64(uint64_t* __restrict__ p, int64_t count, uint64_t value) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

// Zeroes two ranges in one launch (an output and the work-queue counters).
__global__ void k_zero2(uint64_t* __restrict__ a, int64_t na, uint64_t* __restrict__ b, int64_t nb) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < na) a[i] = 0;
  else if (i - na < nb) b[i - na] = 0;
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

cs_status launch_zero2(uint64_t* a, int64_t na, uint64_t* b, int64_t nb, hipStream_t st) {
  if (na + nb <= 0) return CS_OK;
  hipLaunchKernelGGL(k_zero2, dim3((unsigned)ceil_div(na + nb, 256)), dim3(256), 0, st, a, na, b, nb);
  CS_LAUNCH_CHECK();
  return CS_OK;
}

cs_status launch_fill_u64(uint64_t* p, int64_t count, uint64_t value, hipStream_t st) {
  if (count <= 0) return CS_OK;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, st, p, count,
                     value);
  CS_LAUNCH_CHECK();
  return CS_OK;
}

size_t histogram_ws_bytes(int64_t, int) { return 256; }

template <int WM, bool FP4, int EPI = 0>
cs_status launch_mfma(const uint64_t* bits, int64_t n, int64_t ld, uint64_t* hist,
                      unsigned int* ctr, hipStream_t st, FieldArgs f = FieldArgs{}) {
  constexpr int BM = 2 * WM * 32;
  const int64_t T = ceil_div(n, BM);
  const unsigned grid = (unsigned)std::min<int64_t>(T * (T + 1) / 2, device_cu_count());
  hipLaunchKernelGGL((k_count_mfma<WM, FP4, EPI>), dim3(grid), dim3(kThreads), 0, st, bits, n, ld,
                     (unsigned long long*)hist, ctr, f);
  CS_LAUNCH_CHECK();
  return CS_OK;
}

// out[j] = scale (out[j] - phi[j]): the bracket's -phi(j) and the prefactor K / ell^2.
__global__ void k_field_finish(const double* __restrict__ phi, double* __restrict__ out, int64_t n,
                               double scale) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[j] = __dmul_rn(scale, __dsub_rn(out[j], phi[j]));
}

cs_status launch_histogram(const uint64_t* bits, int64_t n, int64_t ld, int counter, uint64_t* hist,
                           void* ws, hipStream_t st) {
  unsigned int* ctr = (unsigned int*)ws;
  cs_status s = launch_zero2(hist, n - 1, (uint64_t*)ws, 4, st);  // bins, 8 queue counters
  if (s != CS_OK) return s;
  const bool big = n > 4096;  // 256x256 output tiles above 4096 points, 128x128 below
  switch (counter) {
    case CS_COUNT_MFMA:
      return big ? launch_mfma<4, false>(bits, n, ld, hist, ctr, st)
                 : launch_mfma<2, false>(bits, n, ld, hist, ctr, st);
    case CS_COUNT_MFMA_FP4:
      return big ? launch_mfma<4, true>(bits, n, ld, hist, ctr, st)
                 : launch_mfma<2, true>(bits, n, ld, hist, ctr, st);
    default: {
      const int64_t T = ceil_div(n, 128);
      const unsigned grid = (unsigned)std::min<int64_t>(T * (T + 1) / 2, 2 * device_cu_count());
      hipLaunchKernelGGL(k_count_bitset, dim3(grid), dim3(kThreads), 0, st, bits, n, ld,
                         (unsigned long long*)hist, ctr,
                         counter == CS_COUNT_BITSET_DENSE ? -1 : kPairTaskMax);
      CS_LAUNCH_CHECK();
      return CS_OK;
    }
  }
}

size_t field_ws_bytes(int64_t, int) { return 256; }

cs_status launch_dalembertian(const uint64_t* bits, int64_t n, int64_t ld, int counter, int dim,
                              double ell, const double* phi, double* out, void* ws, hipStream_t st) {
  unsigned int* ctr = (unsigned int*)ws;
  // out = +0.0, 8 queue counters
  cs_status s = launch_zero2((uint64_t*)out, n, (uint64_t*)ws, 4, st);
  if (s != CS_OK) return s;
  // Eqs. b2d_local, b3d_local, b4d_local: K / ell^2 [-phi(j) + sum_m c_m sum_{L_m(j)} phi(i)].
  FieldArgs f{phi, out, 0.0, 0.0, 0.0, 0.0};
  double K;
  if (dim == 2) {
    K = 2.0;
    f.c0 = 2.0; f.c1 = -4.0; f.c2 = 2.0;
  } else if (dim == 3) {  // eq. b3d_local
    K = (double)prefactor_c3();
    f.c0 = 1.0; f.c1 = -3.375; f.c2 = 2.25;
  } else {
    K = 4.0 / sqrt(6.0);
    f.c0 = 1.0; f.c1 = -9.0; f.c2 = 16.0; f.c3 = -8.0;
  }
  const bool big = n > 4096;
  if (counter == CS_COUNT_MFMA)
    s = big ? launch_mfma<4, false, 1>(bits, n, ld, nullptr, ctr, st, f)
            : launch_mfma<2, false, 1>(bits, n, ld, nullptr, ctr, st, f);
  else
    s = big ? launch_mfma<4, true, 1>(bits, n, ld, nullptr, ctr, st, f)
            : launch_mfma<2, true, 1>(bits, n, ld, nullptr, ctr, st, f);
  if (s != CS_OK) return s;
  hipLaunchKernelGGL(k_field_finish, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, phi, out, n,
                     K / (ell * ell));
  CS_LAUNCH_CHECK();
  return CS_OK;
}

cs_status launch_count_batch(const BatchTile& cfg, bool fp4, const uint64_t* bits,
                             const BatchInst* inst, const uint32_t* items,
                             const BatchQueues& queues, uint64_t* hist, unsigned int* counter,
                             hipStream_t st) {
  const int64_t nitems = queues.off[kBatchQueues];
  if (nitems <= 0) return CS_OK;
  const int mode = cfg.mode;
  const int cus = device_cu_count();
  const int per_cu = mode == 4 ? 1 : (cfg.per_cu == 1 ? 1 : 2);
  const int pair_max = cfg.pair_max < 0 ? -1 : std::min(cfg.pair_max, kPairTaskMax);
  const unsigned grid = (unsigned)std::min<int64_t>(nitems, (int64_t)cus * per_cu);
  unsigned long long* h = (unsigned long long*)hist;
#define CS_BATCH_LAUNCH(M, F)                                                                  \
  hipLaunchKernelGGL((k_count_batch<M, F>), dim3(grid), dim3(kThreads), 0, st, bits, inst, \
                     items, queues, h, counter, pair_max)
  if (mode == 0) CS_BATCH_LAUNCH(0, false);
  else if (mode == 2 && !fp4) CS_BATCH_LAUNCH(2, false);
  else if (mode == 4 && !fp4) CS_BATCH_LAUNCH(4, false);
  else if (mode == 2 && fp4) CS_BATCH_LAUNCH(2, true);
  else if (mode == 4 && fp4) CS_BATCH_LAUNCH(4, true);
  else return CS_ERR_UNSUPPORTED;
#undef CS_BATCH_LAUNCH
  CS_LAUNCH_CHECK();
  return CS_OK;
}

}  // namespace cs
