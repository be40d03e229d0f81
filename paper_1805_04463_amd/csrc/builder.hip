// Causal-matrix builder: writes the symmetric packed bitset S = C + C^T of n
// time-ordered points (Sec. 3.2 "Data Structures for Graphs": a topologically
// sorted DAG kept as P + P^T; Ch. 4: i ≺ j iff timelike separated).
//
// Work decomposition: one wave per 64x64 block (bi <= bj) of the upper triangle.
// Lane l owns column j = 64*bj + l (coordinates in registers); the wave walks the
// 64 rows i of block bi with i's coordinates as wave-uniform (scalar) operands.
// Each predicate is evaluated once per unordered pair:
//   - the wave ballot over lanes is row i's 64-bit word for column block bj;
//   - each lane ORs bit (i - 64*bi) into its own register, which after the loop is
//     row j's word for column block bi (the transposed word), so no second pass.
// Both words are then stored by the lanes that own them.  Four waves of a workgroup
// take four consecutive column blocks of the same row block, so each row i receives
// 32 contiguous bytes from one workgroup.
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

// a ≺ b for a earlier than b in time order.
__device__ inline bool precedes(const Pt<CS_MINK2_DIAMOND>& a, const Pt<CS_MINK2_DIAMOND>& b) {
  return a.u < b.u && a.v < b.v;
}
__device__ inline bool precedes(const Pt<CS_MINK4_DIAMOND>& a, const Pt<CS_MINK4_DIAMOND>& b) {
  double dt = __dsub_rn(b.t, a.t);
  double dx = __dsub_rn(b.x, a.x);
  double dy = __dsub_rn(b.y, a.y);
  double dz = __dsub_rn(b.z, a.z);
  double s = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
  s = __dadd_rn(s, __dmul_rn(dz, dz));
  return dt > 0.0 && __dmul_rn(dt, dt) > s;
}
__device__ inline bool precedes(const Pt<CS_DS4_SLAB>& a, const Pt<CS_DS4_SLAB>& b) {
  // eta_a < eta_b and cos(eta_b - eta_a) < n_a . n_b (both angles in [0, pi]).
  double cd = __dadd_rn(__dmul_rn(a.c, b.c), __dmul_rn(a.s, b.s));
  double dot = __dadd_rn(__dmul_rn(a.n0, b.n0), __dmul_rn(a.n1, b.n1));
  dot = __dadd_rn(dot, __dmul_rn(a.n2, b.n2));
  dot = __dadd_rn(dot, __dmul_rn(a.n3, b.n3));
  return a.x < b.x && cd < dot;
}

constexpr int kWavesPerBlock = 4;

// One wave: the 64x64 block (bi, bj), bi <= bj, of an n-point matrix S with stride ld.
// The wave owning the last column block of a row block also zeroes that row block's
// padding words [nb, ld), so every word of S is written exactly once.
template <int R>
__device__ inline void build_block(const double* __restrict__ coords, int64_t n,
                                   uint64_t* __restrict__ S, int64_t ld, int64_t nb, int64_t bi,
                                   int64_t bj) {
  const int lane = threadIdx.x & 63;
  const int64_t j = bj * 64 + lane;
  const bool jv = j < n;
  Pt<R> pj = load_pt(coords, n, jv ? j : n - 1, (Pt<R>*)nullptr);
  const int64_t i0 = bi * 64;
  const int rows = (int)(n - i0 < 64 ? n - i0 : 64);
  uint64_t rowword = 0, colword = 0;
  for (int r = 0; r < rows; ++r) {
    const int64_t i = i0 + r;
    Pt<R> pi = load_pt(coords, n, i, (Pt<R>*)nullptr);
    const bool rel = jv && i < j && precedes(pi, pj);
    const uint64_t m = __ballot(rel);
    if (lane == r) rowword = m;
    if (rel) colword |= 1ull << r;
  }
  const int64_t irow = i0 + lane;
  if (bi == bj) {
    if (irow < n) S[irow * ld + bi] = rowword | colword;
  } else {
    if (irow < n) S[irow * ld + bj] = rowword;
    if (jv) S[j * ld + bi] = colword;
  }
  if (bj == nb - 1 && irow < n)
    for (int64_t w = nb; w < ld; ++w) S[irow * ld + w] = 0;
}

template <int R>
__global__ __launch_bounds__(256) void k_build(const double* __restrict__ coords, int64_t n,
                                               uint64_t* __restrict__ S, int64_t ld, int64_t nb) {
  const int64_t bi = blockIdx.y;
  const int64_t bj = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (bj >= nb || bj < bi) return;  // wave-uniform exit; no barriers
  build_block<R>(coords, n, S, ld, nb, bi, bj);
}

// Ensemble of 1+1 diamonds: wave w of block b takes work item 4b + w, packed as
// instance << 16 | bi << 8 | bj.
__global__ __launch_bounds__(256) void k_build_batch(const double* __restrict__ coords,
                                                     const BatchInst* __restrict__ inst,
                                                     const uint32_t* __restrict__ items,
                                                     int64_t nitems, uint64_t* __restrict__ bits) {
  const int64_t t = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (t >= nitems) return;
  const uint32_t it = items[t];
  const BatchInst d = inst[it >> 16];
  build_block<CS_MINK2_DIAMOND>(coords + d.coord_off, d.n, bits + d.bits_off, d.ld,
                                ceil_div(d.n, 64), (it >> 8) & 255u, it & 255u);
}

template <int R>
cs_status launch_build(const double* coords, int64_t n, uint64_t* S, int64_t ld, hipStream_t st) {
  const int64_t nb = ceil_div(n, 64);
  dim3 grid((unsigned)ceil_div(nb, kWavesPerBlock), (unsigned)nb);
  hipLaunchKernelGGL(k_build<R>, grid, dim3(64 * kWavesPerBlock), 0, st, coords, n, S, ld, nb);
  CS_LAUNCH_CHECK();
  return CS_OK;
}

}  // namespace

cs_status launch_causal_matrix(int region, const double* coords, int64_t n, uint64_t* bits,
                               int64_t ld, hipStream_t st) {
  switch (region) {
    case CS_MINK2_DIAMOND: return launch_build<CS_MINK2_DIAMOND>(coords, n, bits, ld, st);
    case CS_MINK4_DIAMOND: return launch_build<CS_MINK4_DIAMOND>(coords, n, bits, ld, st);
    case CS_DS4_SLAB: return launch_build<CS_DS4_SLAB>(coords, n, bits, ld, st);
    default: return CS_ERR_UNSUPPORTED;
  }
}

cs_status launch_build_batch(const double* coords, const BatchInst* inst, const uint32_t* items,
                             int64_t nitems, uint64_t* bits, hipStream_t st) {
  if (nitems <= 0) return CS_OK;
  hipLaunchKernelGGL(k_build_batch, dim3((unsigned)ceil_div(nitems, kWavesPerBlock)),
                     dim3(64 * kWavesPerBlock), 0, st, coords, inst, items, nitems, bits);
  CS_LAUNCH_CHECK();
  return CS_OK;
}

}  // namespace cs
