// Causal-matrix builder: writes the symmetric packed bitset S = C + C^T of n
// time-ordered points (Sec. 3.2 "Data Structures for Graphs": a topologically
// sorted DAG kept as P + P^T; Ch. 4: i ≺ j iff timelike separated).
//
// Work decomposition: one wave per 64x64 block (bi <= bj) of the upper triangle.
// Lane l owns row i = 64*bi + l (coordinates in registers) and tests it against the
// 64 column points of block bj, the same for every lane: scalar loads in the 2+1 and
// 3+1 diamonds, staged in LDS elsewhere.  Its 64 answers form row i's word for column
// block bj.  A 64x64 bit transpose across the wave (six butterfly stages of lane
// shuffles) turns those row words into the words of rows j for column block bi, so each
// unordered pair is tested once and both halves of the symmetric matrix are written.
// Workgroups walk 1024 x 1024-point patches, one XCD per patch (k_build).  The ensemble
// builder gives each wave several row blocks against one column block, so that each
// column point read from LDS serves several rows of a lane.
//
// Arithmetic: fp64, in the order written, no contraction (built with
// -ffp-contract=off and explicit round-to-nearest intrinsics); on CDNA4 fp64 VALU
// runs at the rate of non-packed fp32, so no fp32 prefilter is used.
#include "common.h"

namespace cs {
namespace {

template <int R>
struct Pt;
template <>
struct Pt<CS_MINK2_DIAMOND> {
  double u, v;
};
template <>
struct Pt<CS_MINK4_DIAMOND> {
  double t, x, y, z;
};
template <>
struct Pt<CS_DS4_SLAB> {
  double x, c, s, n0, n1, n2, n3;
};
template <>
struct Pt<CS_DS2_SLAB> {
  double eta, th;
};
template <>
struct Pt<CS_MINK3_DIAMOND> {
  double t, x, y;
};

__device__ inline Pt<CS_MINK2_DIAMOND> load_pt(const double* c, int64_t n, int64_t i,
                                               Pt<CS_MINK2_DIAMOND>*) {
  return {c[i], c[n + i]};
}
__device__ inline Pt<CS_MINK4_DIAMOND> load_pt(const double* c, int64_t n, int64_t i,
                                               Pt<CS_MINK4_DIAMOND>*) {
  return {c[i], c[n + i], c[2 * n + i], c[3 * n + i]};
}
__device__ inline Pt<CS_DS4_SLAB> load_pt(const double* c, int64_t n, int64_t i,
                                          Pt<CS_DS4_SLAB>*) {
  return {c[i], c[n + i], c[2 * n + i], c[3 * n + i], c[4 * n + i], c[5 * n + i], c[6 * n + i]};
}

__device__ inline Pt<CS_DS2_SLAB> load_pt(const double* c, int64_t n, int64_t i,
                                          Pt<CS_DS2_SLAB>*) {
  return {c[n + i], c[2 * n + i]};
}
__device__ inline Pt<CS_MINK3_DIAMOND> load_pt(const double* c, int64_t n, int64_t i,
                                               Pt<CS_MINK3_DIAMOND>*) {
  return {c[i], c[n + i], c[2 * n + i]};
}

// a ≺ b for a earlier than b in time order.
__device__ inline bool precedes(const Pt<CS_MINK2_DIAMOND>& a, const Pt<CS_MINK2_DIAMOND>& b) {
  return (a.u < b.u) & (a.v < b.v);
}
__device__ inline bool precedes(const Pt<CS_MINK4_DIAMOND>& a, const Pt<CS_MINK4_DIAMOND>& b) {
  double dt = __dsub_rn(b.t, a.t);
  double dx = __dsub_rn(b.x, a.x);
  double dy = __dsub_rn(b.y, a.y);
  double dz = __dsub_rn(b.z, a.z);
  double s = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
  s = __dadd_rn(s, __dmul_rn(dz, dz));
  return (dt > 0.0) & (__dmul_rn(dt, dt) > s);
}
__device__ inline bool precedes(const Pt<CS_DS4_SLAB>& a, const Pt<CS_DS4_SLAB>& b) {
  // eta_a < eta_b and cos(eta_b - eta_a) < n_a . n_b (both angles in [0, pi]).
  double cd = __dadd_rn(__dmul_rn(a.c, b.c), __dmul_rn(a.s, b.s));
  double dot = __dadd_rn(__dmul_rn(a.n0, b.n0), __dmul_rn(a.n1, b.n1));
  dot = __dadd_rn(dot, __dmul_rn(a.n2, b.n2));
  dot = __dadd_rn(dot, __dmul_rn(a.n3, b.n3));
  return (a.x < b.x) & (cd < dot);
}
__device__ inline bool precedes(const Pt<CS_MINK3_DIAMOND>& a, const Pt<CS_MINK3_DIAMOND>& b) {
  double dt = __dsub_rn(b.t, a.t);
  double dx = __dsub_rn(b.x, a.x);
  double dy = __dsub_rn(b.y, a.y);
  return (dt > 0.0) & (__dmul_rn(dt, dt) > __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)));
}
__device__ inline bool precedes(const Pt<CS_DS2_SLAB>& a, const Pt<CS_DS2_SLAB>& b) {
  // The angular separation the short way round, pi - |pi - |theta_a - theta_b||, below
  // the conformal-time separation (fabs is exact; pi is the double nearest pi).
  const double pi = 3.141592653589793;
  double dth = fabs(__dsub_rn(a.th, b.th));
  dth = __dsub_rn(pi, fabs(__dsub_rn(pi, dth)));
  return (a.eta < b.eta) & (dth < __dsub_rn(b.eta, a.eta));
}

// a ≺ b for points a, b with b no earlier than a in time order (the builder only
// asks this).  In the diamonds dt = t_b - t_a >= 0 exactly, and dt * dt > s >= 0 then
// already excludes dt == 0, so the dt > 0 test of precedes() is dropped: the same answer
// with one compare fewer.  The other regions ask precedes() as it stands.
template <int R>
__device__ inline bool later_precedes(const Pt<R>& a, const Pt<R>& b) {
  return precedes(a, b);
}
template <>
__device__ inline bool later_precedes(const Pt<CS_MINK4_DIAMOND>& a,
                                      const Pt<CS_MINK4_DIAMOND>& b) {
  double dt = __dsub_rn(b.t, a.t);
  double dx = __dsub_rn(b.x, a.x);
  double dy = __dsub_rn(b.y, a.y);
  double dz = __dsub_rn(b.z, a.z);
  double s = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
  s = __dadd_rn(s, __dmul_rn(dz, dz));
  return __dmul_rn(dt, dt) > s;
}
template <>
__device__ inline bool later_precedes(const Pt<CS_MINK3_DIAMOND>& a,
                                      const Pt<CS_MINK3_DIAMOND>& b) {
  double dt = __dsub_rn(b.t, a.t);
  double dx = __dsub_rn(b.x, a.x);
  double dy = __dsub_rn(b.y, a.y);
  return __dmul_rn(dt, dt) > __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
}

// The wave's lane mask of later_precedes(a, b).  Where the relation is the AND of two
// compares, each compare writes its lane mask to scalar registers and the masks are
// ANDed there: a ballot of the AND would first turn it into a per-lane value and back
// (two VALU instructions more per pair test).  fcmp predicate 4 is ordered less-than,
// false for NaN like the C operator.
template <int R>
__device__ inline uint64_t precedes_mask(const Pt<R>& a, const Pt<R>& b) {
  return __builtin_amdgcn_ballot_w64(later_precedes(a, b));
}
template <>
__device__ inline uint64_t precedes_mask(const Pt<CS_MINK2_DIAMOND>& a,
                                         const Pt<CS_MINK2_DIAMOND>& b) {
  return __builtin_amdgcn_fcmp(a.u, b.u, 4) & __builtin_amdgcn_fcmp(a.v, b.v, 4);
}
template <>
__device__ inline uint64_t precedes_mask(const Pt<CS_DS4_SLAB>& a, const Pt<CS_DS4_SLAB>& b) {
  double cd = __dadd_rn(__dmul_rn(a.c, b.c), __dmul_rn(a.s, b.s));
  double dot = __dadd_rn(__dmul_rn(a.n0, b.n0), __dmul_rn(a.n1, b.n1));
  dot = __dadd_rn(dot, __dmul_rn(a.n2, b.n2));
  dot = __dadd_rn(dot, __dmul_rn(a.n3, b.n3));
  return __builtin_amdgcn_fcmp(a.x, b.x, 4) & __builtin_amdgcn_fcmp(cd, dot, 4);
}
template <>
__device__ inline uint64_t precedes_mask(const Pt<CS_DS2_SLAB>& a, const Pt<CS_DS2_SLAB>& b) {
  const double pi = 3.141592653589793;
  double dth = fabs(__dsub_rn(a.th, b.th));
  dth = __dsub_rn(pi, fabs(__dsub_rn(pi, dth)));
  return __builtin_amdgcn_fcmp(a.eta, b.eta, 4) & __builtin_amdgcn_fcmp(dth, __dsub_rn(b.eta, a.eta), 4);
}

// 2 w + (this lane's bit of the wave mask m): one add with m as the carry-in.
__device__ inline uint32_t shift_in(uint32_t w, uint64_t m) {
  uint32_t r;
  uint64_t carry_out;
  asm("v_addc_co_u32_e64 %0, %1, %2, %2, %3" : "=v"(r), "=s"(carry_out) : "v"(w), "s"(m));
  return r;
}

constexpr int kWavesPerBlock = 4;

// 64x64 bit transpose across a wave: lane l holds word x with bit c = element (l, c);
// afterwards lane c holds bit l = element (l, c).  Six butterfly stages; at stage s the
// off-diagonal s x s sub-blocks are swapped with the partner lane l ^ s.
__device__ inline uint64_t wave_transpose64(uint64_t x) {
  const int lane = threadIdx.x & 63;
  const uint64_t lo_masks[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull,
                                0x00FF00FF00FF00FFull, 0x0F0F0F0F0F0F0F0Full,
                                0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int s = 32 >> k;
    const uint64_t mlo = lo_masks[k], mhi = ~mlo;
    const uint32_t ylo = (uint32_t)__shfl_xor((int)(uint32_t)x, s);
    const uint32_t yhi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), s);
    const uint64_t y = ((uint64_t)yhi << 32) | ylo;
    x = (lane & s) ? ((x & mhi) | ((y & mhi) >> s)) : ((x & mlo) | ((y & mlo) << s));
  }
  return x;
}

// Row words of lane l for the 64 column points j0 .. j0+63, one per row point pi[r]:
// bit c is column c.  Columns enter from the top, 63 first, each compare's wave mask
// shifted in as a carry.  The columns are wave-uniform, and each is read once for all RB
// rows of the lane.  In the 3+1 and 2+1 diamonds they come through scalar loads into
// SGPRs and feed the fp64 operations directly, instead of broadcast reads from LDS (16
// bytes per lane per instruction: the LDS bound of those blocks).  The other regions
// stage them in LDS: the 7-plane de Sitter slab's columns, loaded ahead, do not fit the
// scalar registers, and the two-plane predicates are too short to hide the scalar load
// latency (both measured slower); with several rows per lane a broadcast read serves RB
// rows.  A block that ends past n repeats point n-1 for the missing columns (masked off
// by the caller).
template <int R>
constexpr bool kScalarColumns = R == CS_MINK4_DIAMOND || R == CS_MINK3_DIAMOND;

template <int R, bool FULL, int RB>
__device__ __attribute__((always_inline)) inline void row_words(
    const double* __restrict__ coords, int64_t n, int64_t j0, const Pt<R> (&pi)[RB], Pt<R>* cols,
    uint64_t (&out)[RB]) {
  if constexpr (!kScalarColumns<R>) {
    const int lane = threadIdx.x & 63;
    cols[lane] = load_pt(coords, n, j0 + lane < n ? j0 + lane : n - 1, (Pt<R>*)nullptr);
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): the wave's LDS writes have landed
    __builtin_amdgcn_wave_barrier();
  }
  uint32_t half[RB][2];
#pragma unroll
  for (int h = 1; h >= 0; --h) {
    uint32_t w[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) w[r] = 0;
#pragma unroll
    for (int c = 31; c >= 0; --c) {
      int64_t j = j0 + 32 * h + c;
      if (!FULL) j = j < n ? j : n - 1;
      const Pt<R> q = kScalarColumns<R> ? load_pt(coords, n, j, (Pt<R>*)nullptr) : cols[32 * h + c];
#pragma unroll
      for (int r = 0; r < RB; ++r)
        w[r] = shift_in(w[r], precedes_mask(pi[r], q));
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) half[r][h] = w[r];
  }
  if constexpr (!kScalarColumns<R>) __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int r = 0; r < RB; ++r) out[r] = ((uint64_t)half[r][1] << 32) | half[r][0];
}

// One wave: the 64x64 blocks (bi0 + r, bj0 + c), r < RB, c < CB, of an n-point matrix S
// with stride ld, those with bi0 + r <= bj0 + c < nb (bi0 <= bj0; both wave-uniform).
// Lane l owns rows i = 64 (bi0 + r) + l and collects their row words for the 64 column
// points of each block bj0 + c.  The transposed words (rows of block bj0 + c, columns of
// block bi0 + r) come from a 64x64 bit transpose of each row word, so each unordered pair
// is tested once.  Blocks below the diagonal are tested but not written.  The wave owning
// the last column block of a row block also zeroes that row block's padding words
// [nb, ld), so every word of S is written exactly once.
template <int R, int RB, int CB>
__device__ __attribute__((always_inline)) inline void build_block(
    const double* __restrict__ coords, int64_t n, uint64_t* __restrict__ S, int64_t ld, int64_t nb,
    int64_t bi0, int64_t bj0, Pt<R>* cols) {
  const int lane = threadIdx.x & 63;
  Pt<R> pi[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int64_t i = (bi0 + r) * 64 + lane;
    pi[r] = load_pt(coords, n, i < n ? i : n - 1, (Pt<R>*)nullptr);
  }
  uint64_t rows[CB][RB];
  if (bj0 * 64 + 64 <= n) row_words<R, true, RB>(coords, n, bj0 * 64, pi, cols, rows[0]);
  else row_words<R, false, RB>(coords, n, bj0 * 64, pi, cols, rows[0]);
  if constexpr (CB == 2) {
    const int64_t bj = bj0 + 1;
    if (bj < nb) {
      if (bj * 64 + 64 <= n) row_words<R, true, RB>(coords, n, bj * 64, pi, cols, rows[1]);
      else row_words<R, false, RB>(coords, n, bj * 64, pi, cols, rows[1]);
    }
  }
  if constexpr (RB == 4) {
    if (bi0 + RB - 1 < bj0 && bj0 + CB - 1 < nb) {
      // Every block lies above the diagonal and every row is valid: a lane's four
      // transposed words of row j (column blocks bi0 .. bi0 + 3) are contiguous and 16-byte
      // aligned (bi0 is a multiple of 4, rows start on 64-byte boundaries), and so are its
      // two row words of row i with two column blocks (bj0 even), so they go out as 16-byte
      // stores instead of 8-byte ones.
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const int64_t ncols = n - (bj0 + c) * 64;  // valid columns of the block (>= 1)
        if (ncols < 64)
#pragma unroll
          for (int r = 0; r < RB; ++r) rows[c][r] &= (1ull << ncols) - 1ull;
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int64_t i = (bi0 + r) * 64 + lane;
        if constexpr (CB == 2)
          *(uint4*)(S + i * ld + bj0) = make_uint4((uint32_t)rows[0][r], (uint32_t)(rows[0][r] >> 32),
                                                   (uint32_t)rows[1][r], (uint32_t)(rows[1][r] >> 32));
        else
          S[i * ld + bj0] = rows[0][r];
        if (bj0 + CB - 1 == nb - 1)
          for (int64_t w = nb; w < ld; ++w) S[i * ld + w] = 0;
      }
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        uint64_t cw[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) cw[r] = wave_transpose64(rows[c][r]);
        const int64_t j = (bj0 + c) * 64 + lane;
        if (j < n) {
          uint4* dst = (uint4*)(S + j * ld + bi0);
          dst[0] = make_uint4((uint32_t)cw[0], (uint32_t)(cw[0] >> 32), (uint32_t)cw[1], (uint32_t)(cw[1] >> 32));
          dst[1] = make_uint4((uint32_t)cw[2], (uint32_t)(cw[2] >> 32), (uint32_t)cw[3], (uint32_t)(cw[3] >> 32));
        }
      }
      return;
    }
  }
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    const int64_t bj = bj0 + c;
    if (c > 0 && bj >= nb) break;
    const int64_t j = bj * 64 + lane;
    const bool jv = j < n;
    const int64_t ncols = n - bj * 64;  // valid columns of this block (>= 1)
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int64_t bi = bi0 + r;
      if (bi > bj) break;  // this and the later row blocks lie below the diagonal
      const int64_t i = bi * 64 + lane;
      const bool iv = i < n;
      uint64_t row = rows[c][r];
      if (ncols < 64) row &= (1ull << ncols) - 1ull;
      if (bi == bj) row &= lane == 63 ? 0ull : (~0ull << (lane + 1));  // only j > i
      if (!iv) row = 0;
      const uint64_t col = wave_transpose64(row);  // lane l: row j's bits for columns of bi
      if (bi == bj) {
        if (iv) S[i * ld + bi] = row | col;
      } else {
        if (iv) S[i * ld + bj] = row;
        if (jv) S[j * ld + bi] = col;
      }
      if (bj == nb - 1 && iv)
        for (int64_t w = nb; w < ld; ++w) S[i * ld + w] = 0;
    }
  }
}

// Patches of 16 x 16 blocks (1024 x 1024 points) of the upper triangle, 64 / RB workgroups
// each (16 / RB groups of RB block rows x 4 groups of 4 block columns; a wave takes RB row
// blocks against one column block).  Workgroups are dealt to the 8
// XCDs in turn, so the workgroups of patch p get ids 8 apart: a patch is built
// inside one XCD, whose L2 then holds every 128-byte line of its row segments and of
// its transposed segments until the line is complete, instead of sending partial lines
// from several L2s to HBM.  Below 8 patches (n <= 3072) they are not dealt: the grid is
// the patches' own workgroups.  Patch p counts row-major over the patches (py, px >= py).
#ifndef CS_BUILD_PATCH
#define CS_BUILD_PATCH 16
#endif
constexpr int kPatch = CS_BUILD_PATCH;                       // blocks per patch side
constexpr int kGroups = kPatch / kWavesPerBlock;             // column groups per patch
template <int RB>
constexpr int kPatchWgs = kPatch / RB * kGroups;             // workgroups per patch
// Row blocks per wave, from 8 patches up (n > 3072: below that, the fewer, longer waves
// cost more latency than they save): four, so that each column point read from LDS (or
// loaded into SGPRs) serves four rows of a lane.
template <int R>
constexpr int kRowBlocks = 4;

__device__ inline int64_t patch_row_start(int64_t r, int64_t P) { return r * P - r * (r - 1) / 2; }

template <int R, int RB>
__global__ __launch_bounds__(256) void k_build(const double* __restrict__ coords, int64_t n,
                                               uint64_t* __restrict__ S, int64_t ld, int64_t nb,
                                               int64_t P, int64_t npatch) {
  constexpr int PW = kPatchWgs<RB>;
  __shared__ Pt<R> cols[kScalarColumns<R> ? 1 : kWavesPerBlock][64];
  const int64_t g = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  const bool dealt = npatch >= 8;
  const int64_t p = dealt ? (g / (8 * PW)) * 8 + (g & 7) : g / PW;
  if (p >= npatch) return;
  const int l = (int)(dealt ? (g >> 3) % PW : g % PW);
  // smaller root of r^2 - (2P+1) r + 2p = 0, then exact correction
  const double s2 = 2.0 * (double)P + 1.0;
  int64_t py = (int64_t)((s2 - sqrt(s2 * s2 - 8.0 * (double)p)) * 0.5);
  while (py > 0 && patch_row_start(py, P) > p) --py;
  while (patch_row_start(py + 1, P) <= p) ++py;
  const int64_t px = py + (p - patch_row_start(py, P));
  const int64_t bi = py * kPatch + RB * (l / kGroups);
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t bj = (px * kGroups + l % kGroups) * kWavesPerBlock + wave;
  if (bi >= nb || bj >= nb || bj < bi) return;  // wave-uniform exit; no block barriers below
  build_block<R, RB, 1>(coords, n, S, ld, nb, bi, bj, cols[kScalarColumns<R> ? 0 : wave]);
}

// Ensemble of 1+1 diamonds.  Work items are packed as instance << 16 | g << 8 | bj0: row
// blocks kBuildRowBlocks g + r against column blocks bj0 + c, c < kBuildColBlocks, with
// bj0 >= kBuildRowBlocks g a multiple of kBuildColBlocks.  Each column point read from LDS
// serves kBuildRowBlocks rows of the lane, which takes the blocks off the LDS bound of one
// row per lane, and the words of whole groups leave in 16-byte stores.  The items form kBatchQueues lists of
// equal length (one per XCD, padded with kNoBuildItem); wave w of workgroup b takes
// entry kBuildWaves (b div kBatchQueues) + w of list b mod kBatchQueues.
static_assert(kWavesPerBlock == kBuildWaves, "ensemble builder lists are dealt per workgroup");
__global__ __launch_bounds__(256) void k_build_batch(const double* __restrict__ coords,
                                                     const BatchInst* __restrict__ inst,
                                                     const uint32_t* __restrict__ items,
                                                     int64_t nitems, uint64_t* __restrict__ bits) {
  __shared__ Pt<CS_MINK2_DIAMOND> cols[kWavesPerBlock][64];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t per_list = nitems / kBatchQueues;
  const int64_t t = (int64_t)(blockIdx.x % kBatchQueues) * per_list +
                    (int64_t)(blockIdx.x / kBatchQueues) * kWavesPerBlock + wave;
  const uint32_t it = items[t];
  if (it == kNoBuildItem) return;
  const BatchInst d = inst[it >> 16];
  build_block<CS_MINK2_DIAMOND, kBuildRowBlocks, kBuildColBlocks>(
      coords + d.coord_off, d.n, bits + d.bits_off, d.ld, ceil_div(d.n, 64),
      (int64_t)((it >> 8) & 255u) * kBuildRowBlocks, it & 255u, cols[wave]);
}

template <int R, int RB>
cs_status launch_build_rb(const double* coords, int64_t n, uint64_t* S, int64_t ld, int64_t nb,
                          int64_t P, int64_t npatch, hipStream_t st) {
  // Grid rows of at most 64 rounds of 8 patches: a row stays far below 2^32 work-items.
  constexpr int PW = kPatchWgs<RB>;
  const int64_t rounds = ceil_div(npatch, 8);  // nb <= 65535: at most 2^20 rounds
  const dim3 grid = npatch >= 8 ? dim3((unsigned)(8 * PW * std::min<int64_t>(rounds, 64)),
                                       (unsigned)ceil_div(rounds, 64))
                                : dim3((unsigned)(PW * npatch));
  hipLaunchKernelGGL((k_build<R, RB>), grid, dim3(64 * kWavesPerBlock), 0, st, coords, n, S, ld, nb,
                     P, npatch);
  CS_LAUNCH_CHECK();
  return CS_OK;
}

template <int R>
cs_status launch_build(const double* coords, int64_t n, uint64_t* S, int64_t ld, hipStream_t st) {
  const int64_t nb = ceil_div(n, 64);
  const int64_t P = ceil_div(nb, kPatch), npatch = P * (P + 1) / 2;
  if (kRowBlocks<R> > 1 && npatch >= 8)
    return launch_build_rb<R, kRowBlocks<R>>(coords, n, S, ld, nb, P, npatch, st);
  return launch_build_rb<R, 1>(coords, n, S, ld, nb, P, npatch, st);
}

}  // namespace

cs_status launch_causal_matrix(int region, const double* coords, int64_t n, uint64_t* bits,
                               int64_t ld, hipStream_t st) {
  switch (region) {
    case CS_MINK2_DIAMOND: return launch_build<CS_MINK2_DIAMOND>(coords, n, bits, ld, st);
    case CS_MINK4_DIAMOND: return launch_build<CS_MINK4_DIAMOND>(coords, n, bits, ld, st);
    case CS_DS4_SLAB: return launch_build<CS_DS4_SLAB>(coords, n, bits, ld, st);
    case CS_DS2_SLAB: return launch_build<CS_DS2_SLAB>(coords, n, bits, ld, st);
    case CS_MINK3_DIAMOND: return launch_build<CS_MINK3_DIAMOND>(coords, n, bits, ld, st);
    default: return CS_ERR_UNSUPPORTED;
  }
}

cs_status launch_build_batch(const double* coords, const BatchInst* inst, const uint32_t* items,
                             int64_t nitems, uint64_t* bits, hipStream_t st) {
  if (nitems <= 0) return CS_OK;
  if (nitems % (kBatchQueues * kWavesPerBlock) != 0) return CS_ERR_INVALID_ARG;
  hipLaunchKernelGGL(k_build_batch, dim3((unsigned)(nitems / kWavesPerBlock)),
                     dim3(64 * kWavesPerBlock), 0, st, coords, inst, items, nitems, bits);
  CS_LAUNCH_CHECK();
  return CS_OK;
}

}  // namespace cs
