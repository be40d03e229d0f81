// Shared device helpers of the gfx950 causal-set library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/causal.h"

namespace cs {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Counter-based SplitMix64 (Steele, Lea & Flood 2014).  Output c of a generator
// whose state is s is mix(s + (c+1) * golden), i.e. the published next() called
// c+1 times.  A stream key is output `stream` of the generator seeded with
// output 0 of the generator seeded with `seed`.
// ---------------------------------------------------------------------------
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t sm_output(uint64_t state, uint64_t c) {
  return sm_mix(state + (c + 1) * kGolden);
}
__host__ __device__ inline uint64_t sm_stream_key(uint64_t seed, uint64_t stream) {
  return sm_output(sm_output(seed, 0), stream);
}
__device__ inline double unit53(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }

// Streams of the generator per region.
enum : uint64_t {
  kStreamMink2 = 0,
  kStreamMink4 = 1,
  kStreamDsTime = 2,
  kStreamDsSphere = 3,
  kStreamDs2 = 4,
  kStreamMink3 = 5
};

// Rejection sampling of the S^3 direction gives up after this many tries (probability
// 0.69^4096: never reached in practice, but every loop has a bound).
constexpr int kSphereTries = 4096;

// Bitonic sort element: (key, generation index), ordered lexicographically.
__device__ inline bool key_less(uint64_t ka, uint32_t ga, uint64_t kb, uint32_t gb) {
  return ka < kb || (ka == kb && ga < gb);
}

// Monotone map double -> uint64 (unsigned order equals numeric order).
__device__ inline uint64_t order_bits(double x) {
  uint64_t b = (uint64_t)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

inline int64_t ld_words(int64_t n) { return ((n + 511) / 512) * 8; }
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Coordinate planes per region (2, 4, 7).
inline int coord_planes(int region) {
  switch (region) {
    case CS_MINK2_DIAMOND: return 2;
    case CS_MINK4_DIAMOND: return 4;
    case CS_DS4_SLAB: return 7;
    case CS_DS2_SLAB: return 3;
    case CS_MINK3_DIAMOND: return 3;
    default: return -1;
  }
}

#define CS_HIP_CHECK(expr)                      \
  do {                                          \
    hipError_t _e = (expr);                     \
    if (_e != hipSuccess) return CS_ERR_HIP;    \
  } while (0)

#define CS_LAUNCH_CHECK()                                   \
  do {                                                      \
    hipError_t _e = hipGetLastError();                      \
    if (_e != hipSuccess) return CS_ERR_HIP;                \
  } while (0)

// One instance of an ensemble: size, row stride (uint64 words) and offsets of its
// coordinates (doubles), matrix (uint64 words) and histogram (uint64 bins) in the
// concatenated buffers.
struct BatchInst {
  int64_t n, ld, coord_off, bits_off, hist_off;
};

// Largest instance of an ensemble (its whole histogram fits the LDS bins, its sort
// fits one workgroup's LDS).
constexpr int64_t kBatchMaxN = 8192;
// Ensemble builder: row and column blocks of 64 points per work item, blocks per patch
// side, waves per workgroup, and the padding entry of its per-XCD item lists.
constexpr int kBuildRowBlocks = 4;
constexpr int kBuildColBlocks = 2;
constexpr int kBuildPatch = 16;
constexpr int kBuildWaves = 4;
constexpr uint32_t kNoBuildItem = 0xFFFFFFFFu;

// ---------------------------------------------------------------------------
// Internal launchers (each returns CS_OK or CS_ERR_HIP).
// ---------------------------------------------------------------------------
size_t sprinkle_ws_bytes(int region, int64_t n);
cs_status launch_sprinkle(int region, double eta0, uint64_t seed, int64_t n, double* coords,
                          void* ws, hipStream_t st);
cs_status launch_causal_matrix(int region, const double* coords, int64_t n, uint64_t* bits,
                               int64_t ld, hipStream_t st);
size_t histogram_ws_bytes(int64_t n, int counter);
size_t field_ws_bytes(int64_t n, int counter);
long double prefactor_c3();  // (pi / (3 sqrt 2))^(2/3) / Gamma(5/3), the 2+1 constant
cs_status launch_dalembertian(const uint64_t* bits, int64_t n, int64_t ld, int counter, int dim,
                              double ell, const double* phi, double* out, void* ws, hipStream_t st);
cs_status launch_histogram(const uint64_t* bits, int64_t n, int64_t ld, int counter,
                           uint64_t* hist, void* ws, hipStream_t st);
cs_status launch_action(const uint64_t* hist, int64_t n, int dim, double eps, double* out,
                        hipStream_t st);
cs_status launch_fill_u64(uint64_t* p, int64_t count, uint64_t value, hipStream_t st);
size_t chain_ws_bytes(int64_t n, int64_t count);
// Blocks until the rounds are done (reads a per-round progress count back).
cs_status launch_longest_chain(const uint64_t* bits, int64_t n, int64_t ld, const int64_t* lo,
                               const int64_t* hi, int64_t count, int32_t* length,
                               int32_t* height, void* ws, hipStream_t st);
cs_status launch_degrees(const uint64_t* bits, int64_t n, int64_t ld, int64_t* indeg,
                         int64_t* outdeg, hipStream_t st);
int device_cu_count();

// Allocation-free entry points: bytes of the per-device static scratch array, and its
// device address on the current device (looked up once per device).
constexpr size_t kScratchBytes = 16384;
cs_status scratch_for_current_device(void** out);

// Ensemble pieces (1+1 diamonds).
cs_status launch_sprinkle_batch(const uint64_t* seeds, const BatchInst* inst, int64_t count,
                                double* coords, uint64_t* hist, uint64_t* zero, int nzero,
                                hipStream_t st);
cs_status launch_build_batch(const double* coords, const BatchInst* inst,
                             const uint32_t* items, int64_t nitems, uint64_t* bits,
                             hipStream_t st);
// Launch configuration of an ensemble counter: mode 0 is the bitset counter (128 tiles;
// tiles with more than pair_max related-pair tasks take the dense product, pair_max < 0:
// every tile), modes 2 / 4 the MFMA counter with 128 / 256 tiles on the int8 or (fp4 =
// true) the fp4 matrix cores; per_cu persistent workgroups per compute unit (1 or 2; the
// 256 tiles fit one).
struct BatchTile {
  int mode;
  int per_cu;
  int pair_max;
};
// An ensemble counter's work list in one queue per XCD: queue x is items[off[x] .. off[x+1]).
constexpr int kBatchQueues = 8;
struct BatchQueues {
  uint32_t off[kBatchQueues + 1];
};
// counter: kBatchQueues work counters, zero at launch.
cs_status launch_count_batch(const BatchTile& cfg, bool fp4, const uint64_t* bits,
                             const BatchInst* inst, const uint32_t* items,
                             const BatchQueues& queues, uint64_t* hist, unsigned int* counter,
                             hipStream_t st);
cs_status launch_action_batch(const uint64_t* hist, const BatchInst* inst, int64_t count,
                              int dim, const double* eps, int n_eps, double* out,
                              hipStream_t st);

}  // namespace cs
