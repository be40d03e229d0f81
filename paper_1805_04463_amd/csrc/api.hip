// extern "C" entry points of libcausal.so: argument validation, workspace checks,
// then the internal launchers.  Declarations and the contract are in include/causal.h.
#include <math.h>

#include "common.h"

using namespace cs;

namespace {

constexpr int64_t kMaxN = (int64_t)1 << 31;
// MFMA counters: a 256-row panel (256 * ld_words * 8 bytes) stays below 1 GiB, so panel
// offsets fit the buffer descriptors' 32-bit range with room for out-of-range requests.
constexpr int64_t kMaxMfmaLd = (int64_t)1 << 19;

// fp4 histogram: its accumulators start at 2^23 and hold 2^23 + count exactly while
// counts (at most n - 2) stay below 2^23.
constexpr int64_t kMaxFp4HistN = ((int64_t)1 << 23) + 2;

// Longest chains: one grid row per pair.
constexpr int64_t kMaxChainPairs = 65535;

inline hipStream_t as_stream(void* s) { return (hipStream_t)s; }

inline bool is_mfma(int counter) { return counter == CS_COUNT_MFMA || counter == CS_COUNT_MFMA_FP4; }

cs_status check_n(int64_t n) {
  if (n < 2) return CS_ERR_INVALID_ARG;
  if (n >= kMaxN) return CS_ERR_OVERFLOW;
  return CS_OK;
}

}  // namespace

extern "C" {

int cs_coord_planes(int region) { return coord_planes(region); }

int64_t cs_ld_words(int64_t n) { return n < 0 ? -1 : ld_words(n); }

const char* cs_status_string(cs_status s) {
  switch (s) {
    case CS_OK: return "ok";
    case CS_ERR_INVALID_ARG: return "invalid argument";
    case CS_ERR_UNSUPPORTED: return "unsupported region, counter or dimension";
    case CS_ERR_WORKSPACE: return "workspace too small";
    case CS_ERR_OVERFLOW: return "size too large";
    case CS_ERR_HIP: return "HIP runtime error";
    case CS_ERR_NO_DEVICE: return "no gfx950 device";
    default: return "unknown status";
  }
}

size_t cs_sprinkle_workspace_bytes(int region, int64_t n) {
  if (coord_planes(region) < 0 || check_n(n) != CS_OK) return 0;
  return sprinkle_ws_bytes(region, n);
}

cs_status cs_sprinkle(int region, double eta0, uint64_t seed, int64_t n, double* coords,
                      void* workspace, size_t workspace_bytes, void* stream) {
  if (coord_planes(region) < 0) return CS_ERR_UNSUPPORTED;
  cs_status s = check_n(n);
  if (s != CS_OK) return s;
  if (!coords || !workspace) return CS_ERR_INVALID_ARG;
  if ((region == CS_DS4_SLAB || region == CS_DS2_SLAB) &&
      !(eta0 > 0.0 && eta0 < 1.5707963267948966))
    return CS_ERR_INVALID_ARG;
  if (workspace_bytes < sprinkle_ws_bytes(region, n)) return CS_ERR_WORKSPACE;
  return launch_sprinkle(region, eta0, seed, n, coords, workspace, as_stream(stream));
}

cs_status cs_causal_matrix(int region, const double* coords, int64_t n, uint64_t* bits,
                           int64_t ld_words_, void* stream) {
  if (coord_planes(region) < 0) return CS_ERR_UNSUPPORTED;
  cs_status s = check_n(n);
  if (s != CS_OK) return s;
  if (!coords || !bits || ld_words_ < ld_words(n)) return CS_ERR_INVALID_ARG;
  if (ceil_div(n, 64) > 65535) return CS_ERR_OVERFLOW;  // grid rows of 64-point blocks
  return launch_causal_matrix(region, coords, n, bits, ld_words_, as_stream(stream));
}

size_t cs_histogram_workspace_bytes(int64_t n, int counter) {
  if (check_n(n) != CS_OK || counter < CS_COUNT_BITSET || counter > CS_COUNT_BITSET_DENSE) return 0;
  return histogram_ws_bytes(n, counter);
}

cs_status cs_interval_histogram(const uint64_t* bits, int64_t n, int64_t ld_words_, int counter,
                                uint64_t* hist, void* workspace, size_t workspace_bytes,
                                void* stream) {
  if (counter < CS_COUNT_BITSET || counter > CS_COUNT_BITSET_DENSE) return CS_ERR_UNSUPPORTED;
  cs_status s = check_n(n);
  if (s != CS_OK) return s;
  if (!bits || !hist || !workspace || ld_words_ < ld_words(n)) return CS_ERR_INVALID_ARG;
  if (counter == CS_COUNT_MFMA_FP4 && n >= kMaxFp4HistN) return CS_ERR_OVERFLOW;
  if (is_mfma(counter) && ld_words_ > kMaxMfmaLd) return CS_ERR_OVERFLOW;
  if (workspace_bytes < histogram_ws_bytes(n, counter)) return CS_ERR_WORKSPACE;
  return launch_histogram(bits, n, ld_words_, counter, hist, workspace, as_stream(stream));
}

cs_status cs_interval_histogram_noalloc(const uint64_t* bits, int64_t n, int64_t ld_words_,
                                        int counter, uint64_t* hist, void* stream) {
  if (counter < CS_COUNT_BITSET || counter > CS_COUNT_BITSET_DENSE) return CS_ERR_UNSUPPORTED;
  cs_status s = check_n(n);
  if (s != CS_OK) return s;
  if (!bits || !hist || ld_words_ < ld_words(n)) return CS_ERR_INVALID_ARG;
  if (counter == CS_COUNT_MFMA_FP4 && n >= kMaxFp4HistN) return CS_ERR_OVERFLOW;
  if (is_mfma(counter) && ld_words_ > kMaxMfmaLd) return CS_ERR_OVERFLOW;
  if (histogram_ws_bytes(n, counter) > kScratchBytes) return CS_ERR_WORKSPACE;
  void* ws = nullptr;
  s = scratch_for_current_device(&ws);
  if (s != CS_OK) return s;
  return launch_histogram(bits, n, ld_words_, counter, hist, ws, as_stream(stream));
}

size_t cs_dalembertian_workspace_bytes(int64_t n, int counter) {
  if (check_n(n) != CS_OK || (counter != CS_COUNT_MFMA && counter != CS_COUNT_MFMA_FP4)) return 0;
  return field_ws_bytes(n, counter);
}

cs_status cs_dalembertian(const uint64_t* bits, int64_t n, int64_t ld_words_, int dim, double ell,
                          int counter, const double* phi, double* out, void* workspace,
                          size_t workspace_bytes, void* stream) {
  if (dim < 2 || dim > 4) return CS_ERR_UNSUPPORTED;
  if (counter != CS_COUNT_MFMA && counter != CS_COUNT_MFMA_FP4) return CS_ERR_UNSUPPORTED;
  cs_status s = check_n(n);
  if (s != CS_OK) return s;
  if (!bits || !phi || !out || !workspace || ld_words_ < ld_words(n)) return CS_ERR_INVALID_ARG;
  if (!(ell > 0.0) || !isfinite(ell)) return CS_ERR_INVALID_ARG;
  if (counter == CS_COUNT_MFMA_FP4 && n >= (int64_t)1 << 24) return CS_ERR_OVERFLOW;
  if (ld_words_ > kMaxMfmaLd) return CS_ERR_OVERFLOW;
  if (workspace_bytes < field_ws_bytes(n, counter)) return CS_ERR_WORKSPACE;
  return launch_dalembertian(bits, n, ld_words_, counter, dim, ell, phi, out, workspace,
                             as_stream(stream));
}

size_t cs_longest_chain_workspace_bytes(int64_t n, int64_t count) {
  if (check_n(n) != CS_OK || count < 1 || count > kMaxChainPairs) return 0;
  return chain_ws_bytes(n, count);
}

cs_status cs_longest_chain(const uint64_t* bits, int64_t n, int64_t ld_words_, const int64_t* lo,
                           const int64_t* hi, int64_t count, int32_t* length, int32_t* height,
                           void* workspace, size_t workspace_bytes, void* stream) {
  cs_status s = check_n(n);
  if (s != CS_OK) return s;
  if (!bits || !lo || !hi || !length || !workspace || ld_words_ < ld_words(n) || count < 1)
    return CS_ERR_INVALID_ARG;
  if (count > kMaxChainPairs) return CS_ERR_OVERFLOW;
  for (int64_t k = 0; k < count; ++k)
    if (lo[k] < -1 || lo[k] >= n || hi[k] < 0 || hi[k] > n || lo[k] >= hi[k])
      return CS_ERR_INVALID_ARG;
  if (workspace_bytes < chain_ws_bytes(n, count)) return CS_ERR_WORKSPACE;
  return launch_longest_chain(bits, n, ld_words_, lo, hi, count, length, height, workspace,
                              as_stream(stream));
}

cs_status cs_degrees(const uint64_t* bits, int64_t n, int64_t ld_words_, int64_t* indeg,
                     int64_t* outdeg, void* stream) {
  cs_status s = check_n(n);
  if (s != CS_OK) return s;
  if (!bits || (!indeg && !outdeg) || ld_words_ < ld_words(n)) return CS_ERR_INVALID_ARG;
  return launch_degrees(bits, n, ld_words_, indeg, outdeg, as_stream(stream));
}

cs_status cs_action(const uint64_t* hist, int64_t n, int dim, double eps, double* out,
                    void* stream) {
  if (dim < 2 || dim > 4) return CS_ERR_UNSUPPORTED;
  cs_status s = check_n(n);
  if (s != CS_OK) return s;
  if (!hist || !out || !(eps >= 0.0 && eps <= 1.0)) return CS_ERR_INVALID_ARG;
  return launch_action(hist, n, dim, eps, out, as_stream(stream));
}

}  // extern "C"
