// Benincasa-Dowker action from the interval abundances (Sec. 4.2).
//
// Local:    S^(1+1) = 2 (N - 2N_0 + 4N_1 - 2N_2),
//           S^(2+1) = C_3 (N - N_0 + (27/8) N_1 - (9/4) N_2),
//           S^(3+1) = (4/sqrt 6)(N - N_0 + 9N_1 - 16N_2 + 8N_3)      (l = l_p)
// Smeared:  S_eps^(1+1) = 2 eps [N - 2 eps sum_m N_m f_2(m, eps)]
//           S_eps^(2+1) = C_3 eps^(2/3) [N - eps sum_m N_m f_3(m, eps)]
//           S_eps^(3+1) = 4 sqrt(eps/6) [N - eps sum_m N_m f_4(m, eps)]
// with C_3 = (pi / (3 sqrt 2))^(2/3) / Gamma(5/3) and the smearing functions multiplied
// out so no power of (1 - eps) is negative:
//   f_2(m) = (1-e)^(m-2) [(1-e)^2 - 2m e(1-e) + m(m-1)/2 e^2]                m >= 2
//   f_3(m) = (1-e)^(m-2) [(1-e)^2 - (27/8) m e(1-e) + (9/8) m(m-1) e^2]      m >= 2
//   f_4(m) = (1-e)^(m-3) [(1-e)^3 - 9m e(1-e)^2 + 8m(m-1) e^2 (1-e)
//                          - 4 (m(m-1)(m-2)/3) e^3]                          m >= 3
// and the first terms written directly.  The smeared sum is badly conditioned (the
// terms are far larger than the result), so weights and sum are carried in
// double-double (error-free transformations: Knuth's two-sum, Dekker's product via
// fma), then rounded once.  The local combination is an exact 128-bit integer.
//
// One workgroup of 1024 threads per action; bins are dealt in chunks of 8, and the
// walk stops where the weights have fallen below 1e-304.
#include "common.h"

namespace cs {
namespace {

struct dd {
  double hi, lo;
};

__device__ inline dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__device__ inline dd fast_two_sum(double a, double b) {  // |a| >= |b|
  double s = a + b;
  return {s, b - (s - a)};
}
__device__ inline dd two_prod(double a, double b) {
  double p = a * b;
  return {p, fma(a, b, -p)};
}
__device__ inline dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}
__device__ inline dd dd_mul(dd a, dd b) {
  dd p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return fast_two_sum(p.hi, p.lo);
}
__device__ inline dd dd_mul_d(dd a, double b) {
  dd p = two_prod(a.hi, b);
  p.lo += a.lo * b;
  return fast_two_sum(p.hi, p.lo);
}
__device__ inline dd dd_from_u64(uint64_t x) {
  double hi = (double)x;                       // rounded
  int64_t rest = (int64_t)(x - (uint64_t)hi);  // exact remainder, |rest| < 2^11
  return fast_two_sum(hi, (double)rest);
}
__device__ inline dd dd_powi(dd b, int64_t e) {  // e >= 0, 0^0 = 1
  dd r = {1.0, 0.0};
  while (e > 0) {
    if (e & 1) r = dd_mul(r, b);
    b = dd_mul(b, b);
    e >>= 1;
  }
  return r;
}
__device__ inline dd dd_sqrt(dd a) {  // one Newton step from the fp64 root
  if (a.hi <= 0.0) return {0.0, 0.0};
  double s = sqrt(a.hi);
  dd s2 = two_prod(s, s);
  double corr = ((a.hi - s2.hi) - s2.lo + a.lo) / (2.0 * s);
  return fast_two_sum(s, corr);
}

// Bracket polynomials: f(m) = (1-e)^(m-K) * B(m) for m >= K (K = 2, or 3 in 3+1).
struct Smear {
  int dim;
  dd e, q;              // eps and 1 - eps
  dd p[4];              // e^k (1-e)^(K-k), k = 0..K
};

__device__ inline dd bracket(const Smear& s, int64_t m) {
  const double md = (double)m, m1 = (double)(m - 1), m2 = (double)(m - 2);
  if (s.dim == 2) {
    // (1-e)^2 - 2m e(1-e) + (m(m-1)/2) e^2 ; m(m-1)/2 is an integer
    dd c2 = (m % 2 == 0) ? two_prod(md * 0.5, m1) : two_prod(md, m1 * 0.5);
    dd r = s.p[0];
    r = dd_add(r, dd_mul_d(s.p[1], -2.0 * md));
    r = dd_add(r, dd_mul(s.p[2], c2));
    return r;
  }
  if (s.dim == 3) {
    // (1-e)^2 - (27/8) m e(1-e) + (9/8) m(m-1) e^2 ; 27/8 and 9/8 are exact
    dd r = s.p[0];
    r = dd_add(r, dd_mul_d(s.p[1], -3.375 * md));
    r = dd_add(r, dd_mul(s.p[2], dd_mul_d(two_prod(md, m1), 1.125)));
    return r;
  }
  // (1-e)^3 - 9m e(1-e)^2 + 8m(m-1) e^2(1-e) - 4 (m(m-1)(m-2)/3) e^3
  dd c2 = dd_mul_d(two_prod(md, m1), 8.0);
  double a = md, b = m1, c = m2;  // divide the factor that is a multiple of 3
  if (m % 3 == 0) a = md / 3.0; else if ((m - 1) % 3 == 0) b = m1 / 3.0; else c = m2 / 3.0;
  dd c3 = dd_mul_d(dd_mul_d(two_prod(a, b), c), -4.0);
  dd r = s.p[0];
  r = dd_add(r, dd_mul_d(s.p[1], -9.0 * md));
  r = dd_add(r, dd_mul(s.p[2], c2));
  r = dd_add(r, dd_mul(s.p[3], c3));
  return r;
}

// f(m) for the first bins (m < K), from sum_k c_k(m) e^k (1-e)^(m-k).
__device__ inline dd small_weight(const Smear& s, int64_t m) {
  if (m == 0) return {1.0, 0.0};
  if (s.dim == 2) {  // m = 1: (1-e) - 2e
    return dd_add(s.q, dd_mul_d(s.e, -2.0));
  }
  if (s.dim == 3) {  // m = 1: (1-e) - (27/8) e
    return dd_add(s.q, dd_mul_d(s.e, -3.375));
  }
  if (m == 1) return dd_add(s.q, dd_mul_d(s.e, -9.0));  // (1-e) - 9e
  // m = 2: (1-e)^2 - 18 e(1-e) + 16 e^2
  dd r = dd_mul(s.q, s.q);
  r = dd_add(r, dd_mul_d(dd_mul(s.e, s.q), -18.0));
  r = dd_add(r, dd_mul_d(dd_mul(s.e, s.e), 16.0));
  return r;
}

constexpr int kActThreads = 1024;

// The action of one histogram by one workgroup of kActThreads threads.
// c3: for dim 3, the prefactor in double-double (C_3 / 8 for the local action, whose
// bracket is taken times 8 to stay an integer; C_3 eps^(2/3) for the smeared one).
__device__ __attribute__((always_inline)) inline void action_block(
    const uint64_t* __restrict__ hist, int64_t n, int dim, double eps, dd c3,
    double* __restrict__ out, double* s_hi, double* s_lo) {
  const int64_t nb = n - 1;
  if (eps == 0.0) {
    if (threadIdx.x == 0) {
      // the first four bins (absent ones are 0), as scalars: no indexed local array
      const __int128 h0 = (__int128)hist[0];
      const __int128 h1 = nb > 1 ? (__int128)hist[1] : 0;
      const __int128 h2 = nb > 2 ? (__int128)hist[2] : 0;
      const __int128 h3 = nb > 3 ? (__int128)hist[3] : 0;
      const __int128 h[4] = {h0, h1, h2, h3};
      __int128 I;
      if (dim == 2) {
        I = (__int128)n - 2 * h[0] + 4 * h[1] - 2 * h[2];
        out[0] = 2.0 * (double)I;
      } else if (dim == 3) {
        I = 8 * (__int128)n - 8 * h[0] + 27 * h[1] - 18 * h[2];
        double Ihi = (double)I;
        double Ilo = (double)(I - (__int128)Ihi);
        dd r = dd_add(dd_mul_d(c3, Ihi), dd_mul_d(c3, Ilo));
        out[0] = r.hi + r.lo;
      } else {
        I = (__int128)n - h[0] + 9 * h[1] - 16 * h[2] + 8 * h[3];
        // 4/sqrt(6) in double-double times I (I split exactly into two doubles)
        dd c = dd_sqrt(dd{6.0, 0.0});
        // 4 / c by one Newton step on the fp64 quotient
        double q0 = 4.0 / c.hi;
        dd qc = dd_mul_d(c, q0);
        double corr = ((4.0 - qc.hi) - qc.lo) / c.hi;
        dd k = fast_two_sum(q0, corr);
        double Ihi = (double)I;
        double Ilo = (double)(I - (__int128)Ihi);
        dd r = dd_add(dd_mul_d(k, Ihi), dd_mul_d(k, Ilo));
        out[0] = r.hi + r.lo;
      }
    }
    return;
  }
  Smear sm;
  sm.dim = dim;
  sm.e = {eps, 0.0};
  sm.q = two_sum(1.0, -eps);
  const int K = dim == 4 ? 3 : 2;
#pragma unroll
  for (int k = 0; k < 4; ++k)  // constant indices after unrolling (p[3] unused below 3+1)
    sm.p[k] = k <= K ? dd_mul(dd_powi(sm.e, k), dd_powi(sm.q, K - k)) : dd{0.0, 0.0};

  // The weights fall as (1-e)^m: past the bin where (1-e)^(m-K) < e^-700 (about
  // 2^-1010) a term is at most 2^-1010 * 2^93 (bracket, m < 2^31) * 2^61 (count), and all
  // of them together stay below 2^-820, so the walk stops there (near m = 6600 for
  // e = 0.1) instead of covering all n - 1 bins.
  const double log_q = log1p(-eps);  // -inf for eps = 1: only the bins up to K
  int64_t walk = nb;                  // bins up to the cut-off (uniform)
  if (log_q < 0.0) {
    const double cut = (double)K + 700.0 / -log_q + 1.0;
    if (cut < (double)walk) walk = (int64_t)cut;
  }
  // One pass: thread t takes the bins [t C, t C + C) of the walk, with C chosen so that
  // about 512 threads (two waves per SIMD) share it.  Each thread pays once for its first
  // power (1-e)^(m-K), by repeated squaring, then one multiplication per bin, so fewer
  // threads with longer chunks do less work in total, down to that occupancy.
  constexpr int64_t kActBusy = 512;
  const int64_t chunk = walk <= 4 * kActBusy ? 4 : (walk + kActBusy - 1) / kActBusy;
  dd acc = {0.0, 0.0};
  {
    int64_t m = (int64_t)threadIdx.x * chunk;
    const int64_t m1 = m + chunk < walk ? m + chunk : walk;
    for (; m < m1 && m < K; ++m) {
      if (hist[m]) acc = dd_add(acc, dd_mul(dd_from_u64(hist[m]), small_weight(sm, m)));
    }
    if (m < m1) {
      dd pw = dd_powi(sm.q, m - K);  // (1-e)^(m-K)
      for (; m < m1; ++m) {
        const uint64_t h = hist[m];
        if (h) acc = dd_add(acc, dd_mul(dd_from_u64(h), dd_mul(pw, bracket(sm, m))));
        pw = dd_mul(pw, sm.q);
      }
    }
  }
  // Double-double sum over the workgroup: within each wave by lane exchanges, then the
  // waves' partial sums through LDS and one barrier.
  for (int off = 32; off > 0; off >>= 1) {
    const dd o = {__shfl_xor(acc.hi, off), __shfl_xor(acc.lo, off)};
    acc = dd_add(acc, o);
  }
  constexpr int kWaves = kActThreads / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    s_hi[wave] = acc.hi;
    s_lo[wave] = acc.lo;
  }
  __syncthreads();
  if (wave == 0) {
    acc = lane < kWaves ? dd{s_hi[lane], s_lo[lane]} : dd{0.0, 0.0};
    for (int off = kWaves / 2; off > 0; off >>= 1) {
      const dd o = {__shfl_xor(acc.hi, off), __shfl_xor(acc.lo, off)};
      acc = dd_add(acc, o);
    }
  }
  if (threadIdx.x == 0) {
    dd sum = acc;
    dd ec = dim == 2 ? dd{2.0 * eps, 0.0} : dd{eps, 0.0};
    dd br = dd_add(dd{(double)n, 0.0}, dd_mul(dd{-ec.hi, -ec.lo}, sum));
    dd pref;
    if (dim == 2) {
      pref = {2.0 * eps, 0.0};
    } else if (dim == 3) {
      pref = c3;
    } else {
      // eps/6 in double-double (fp64 quotient plus its exact residual / 6), then sqrt
      double q0 = eps / 6.0;
      dd q6 = two_prod(q0, 6.0);
      dd e6 = fast_two_sum(q0, ((eps - q6.hi) - q6.lo) / 6.0);
      pref = dd_mul_d(dd_sqrt(e6), 4.0);
    }
    dd s = dd_mul(pref, br);
    out[0] = s.hi + s.lo;
  }
}

__global__ __launch_bounds__(kActThreads) void k_action(const uint64_t* __restrict__ hist, int64_t n,
                                                        int dim, double eps, double c3hi, double c3lo,
                                                        double* __restrict__ out) {
  __shared__ double s_hi[kActThreads / 64], s_lo[kActThreads / 64];  // per wave
  action_block(hist, n, dim, eps, dd{c3hi, c3lo}, out, s_hi, s_lo);
}

// Ensemble: block k * n_eps + e evaluates eps[e] for instance k.
__global__ __launch_bounds__(kActThreads) void k_action_batch(const uint64_t* __restrict__ hist,
                                                              const BatchInst* __restrict__ inst,
                                                              int dim, const double* __restrict__ eps,
                                                              int n_eps, double* __restrict__ out) {
  __shared__ double s_hi[kActThreads / 64], s_lo[kActThreads / 64];  // per wave
  const int k = blockIdx.x / n_eps, e = blockIdx.x % n_eps;
  const BatchInst d = inst[k];
  action_block(hist + d.hist_off, d.n, dim, eps[e], dd{0.0, 0.0}, out + blockIdx.x, s_hi, s_lo);
}

}  // namespace

long double prefactor_c3() {  // (pi / (3 sqrt 2))^(2/3) / Gamma(5/3), in extended precision
  const long double p = acosl(-1.0L) / (3.0L * sqrtl(2.0L));
  return cbrtl(p * p) / tgammal(5.0L / 3.0L);
}

cs_status launch_action(const uint64_t* hist, int64_t n, int dim, double eps, double* out,
                        hipStream_t st) {
  double c3hi = 0.0, c3lo = 0.0;
  if (dim == 3) {
    const long double c = eps == 0.0 ? prefactor_c3() / 8.0L
                                     : prefactor_c3() * cbrtl((long double)eps * (long double)eps);
    c3hi = (double)c;
    c3lo = (double)(c - (long double)c3hi);
  }
  hipLaunchKernelGGL(k_action, dim3(1), dim3(kActThreads), 0, st, hist, n, dim, eps, c3hi, c3lo,
                     out);
  CS_LAUNCH_CHECK();
  return CS_OK;
}

cs_status launch_action_batch(const uint64_t* hist, const BatchInst* inst, int64_t count, int dim,
                              const double* eps, int n_eps, double* out, hipStream_t st) {
  if (count <= 0 || n_eps <= 0) return CS_OK;
  hipLaunchKernelGGL(k_action_batch, dim3((unsigned)(count * n_eps)), dim3(kActThreads), 0, st, hist,
                     inst, dim, eps, n_eps, out);
  CS_LAUNCH_CHECK();
  return CS_OK;
}

}  // namespace cs
