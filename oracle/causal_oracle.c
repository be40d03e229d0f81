/*
 * causal_oracle.c -- plain, slow, obviously correct CPU oracle for the causal-set
 * interval-abundance path.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the reference the GPU library is checked
 * against.  Only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg may load it.  It shares no code, header, table or constant generator with
 * the GPU library; every definition below is written out from the thesis
 * (W. J. Cunningham, "High Performance Algorithms for Quantum Gravity and
 * Cosmology", 2018) or from the published definition of the generator it uses.
 *
 * What it computes, and where each piece is defined:
 *   sprinkle      App. A, "Causal Set Sprinklings": 1+1 Minkowski diamond
 *                 (u, v uniform), 3+1 Minkowski diamond (here by rejection from the
 *                 bounding box), 3+1 de Sitter slab with spherical foliation
 *                 (density sec^4(eta) in conformal time, uniform on S^3), and the
 *                 1+1 de Sitter slab of the benchmark section (Sec. 4.3: metric
 *                 sec^2(eta)(-d eta^2 + d theta^2), density sec^2(eta), theta
 *                 uniform on the circle), and the 2+1 Minkowski diamond (App. A, here by
 *                 rejection from the bounding box like the 3+1 one).
 *   time order    Sec. 3.2 "Pairwise Relations": elements are labelled so that a
 *                 later index never precedes an earlier one.
 *   causal matrix Ch. 4 introduction: i and j are related when timelike
 *                 separated; stored as P + P^T (Sec. 3.2 "Data Structures").
 *   abundances    the inclusive order intervals (eq. IOIs) and the Alexandroff set
 *                 A_ij = J+(i) ∩ J-(j) (Sec. 2): for every element j and every i in its
 *                 past, the elements of j's past that are also in i's future; the
 *                 quantity of Alg. "Naive Interval Abundance Measurement".
 *   fast tier     Alg. "Optimized Interval Abundance Measurement": word-wise AND
 *                 + popcount over the columns strictly between i and j.
 *   action        Sec. 4.2: local BD actions S^(1+1), S^(3+1) and their smeared
 *                 forms S_eps with the smearing functions f_2 and f_4.
 *   d'Alembertian Sec. 4.1, eqs. b2d_local and b4d_local: B phi(j) from the sums of
 *                 phi over the inclusive order intervals L_1 .. L_4 of each element.
 *   chains        Sec. 2.5.2 "Set Partitions", algorithm "Maximal Chain Length": the
 *                 longest chain between two elements through their Alexandroff set, by
 *                 the memoised recursion from the future element back to the past one;
 *                 per-element heights by the same recursion run from the past end.
 *   degrees       Sec. 3.2 (degree vectors): past and future relations of each element.
 *
 * Parity pins (see tests/test_oracle_*.py): generator test vector, brute-force
 * enumeration of all 2D orders on tiny sets, closed forms (chains, antichains,
 * disjoint chains), exact invariants (sum N_n = R, sum n N_n = sum indeg*outdeg),
 * the numpy C@C special case, statistical moments (ordering fractions 1/4 and
 * 1/10, 4D acceptance pi/24, conformal-time marginals, the 1+1 de Sitter relation
 * probability E|d eta|/pi), symmetries of the cylinder (rotations and reflections
 * of theta), transitivity of the relation, and exact rational evaluation of the
 * smeared sums.
 *
 * Compiled with -O2 -fopenmp -ffp-contract=off: no fused multiply-add, so every
 * floating-point predicate is the exact sequence of IEEE operations written here.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>
#include <quadmath.h>

/* Region codes (same numeric values as the GPU library's public enumeration). */
enum { OR_MINK2_DIAMOND = 0, OR_MINK4_DIAMOND = 1, OR_DS4_SLAB = 2, OR_DS2_SLAB = 3,
       OR_MINK3_DIAMOND = 4 };

/* ------------------------------------------------------------------------- */
/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), as in the public-domain       */
/* reference next(): state += 0x9E3779B97F4A7C15, then the output mix below.   */
/* ------------------------------------------------------------------------- */
static const uint64_t OR_GOLDEN = 0x9E3779B97F4A7C15ULL;

static uint64_t or_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* The published sequential generator: advance the state, return the mix. */
uint64_t or_splitmix64_next(uint64_t *state)
{
    *state += OR_GOLDEN;
    return or_mix(*state);
}

/* Output number c (0-based) of a SplitMix64 generator started at `state`:
 * calling next() c+1 times leaves state + (c+1)*golden, so this is a jump. */
static uint64_t or_output(uint64_t state, uint64_t c)
{
    return or_mix(state + (c + 1) * OR_GOLDEN);
}

/* Stream key: output `stream` of the generator started at output 0 of the
 * generator started at `seed`. */
static uint64_t or_stream_key(uint64_t seed, uint64_t stream)
{
    return or_output(or_output(seed, 0), stream);
}

uint64_t or_draw(uint64_t seed, uint64_t stream, uint64_t c)
{
    return or_output(or_stream_key(seed, stream), c);
}

/* Uniform on [0,1): top 53 bits times 2^-53 (exact). */
static double or_unit(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }

/* ------------------------------------------------------------------------- */
/* Sprinkling                                                                  */
/* ------------------------------------------------------------------------- */

int or_coord_planes(int region)
{
    switch (region) {
    case OR_MINK2_DIAMOND: return 2;  /* u, v                         */
    case OR_MINK4_DIAMOND: return 4;  /* t, x, y, z                   */
    case OR_DS4_SLAB:      return 7;  /* tan eta, cos eta, sin eta, n0..n3 on S^3 */
    case OR_DS2_SLAB:      return 3;  /* tan eta, eta, theta                        */
    case OR_MINK3_DIAMOND: return 3;  /* t, x, y                                    */
    default:               return -1;
    }
}

typedef struct { uint64_t key; int64_t gen; } or_sortkey;

static int or_cmp_key(const void *a, const void *b)
{
    const or_sortkey *x = (const or_sortkey *)a, *y = (const or_sortkey *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->gen != y->gen) return x->gen < y->gen ? -1 : 1;
    return 0;
}

/* Monotone map of a double onto uint64 so that unsigned order = numeric order
 * (negative numbers: all bits flipped; non-negative: sign bit set). */
static uint64_t or_order_bits(double x)
{
    uint64_t b;
    memcpy(&b, &x, sizeof b);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ULL);
}

/*
 * Sprinkle n points into the region and label them in time order.
 * Output: SoA planes, coords[p*n + i] for plane p, sorted.
 * eta0 is used by the de Sitter slab only (eta in [-eta0, eta0]).
 * Returns 0 on success, -1 on bad arguments.
 */
int or_sprinkle(int region, double eta0, uint64_t seed, int64_t n, double *coords)
{
    int planes = or_coord_planes(region);
    if (planes < 0 || n < 1) return -1;
    double *raw = (double *)malloc(sizeof(double) * (size_t)planes * (size_t)n);
    or_sortkey *keys = (or_sortkey *)malloc(sizeof(or_sortkey) * (size_t)n);
    if (!raw || !keys) { free(raw); free(keys); return -1; }

    if (region == OR_MINK2_DIAMOND) {
        /* 1+1 diamond, u0 = v0 = 1: u = U, v = U (App. A).  Time order by the
         * exact integer u+v (scaled by 2^53); a related pair has both u and v
         * larger, hence a strictly larger key. */
        uint64_t s = or_stream_key(seed, 0);
        for (int64_t g = 0; g < n; g++) {
            uint64_t ku = or_output(s, 2 * (uint64_t)g) >> 11;
            uint64_t kv = or_output(s, 2 * (uint64_t)g + 1) >> 11;
            raw[0 * n + g] = (double)ku * 0x1.0p-53;
            raw[1 * n + g] = (double)kv * 0x1.0p-53;
            keys[g].key = ku + kv;
            keys[g].gen = g;
        }
    } else if (region == OR_MINK4_DIAMOND) {
        /* Alexandrov interval of height 1 between (0,0,0,0) and (1,0,0,0):
         * candidates uniform in [0,1) x [-1/2,1/2)^3, accepted when the spatial
         * radius is inside both cones: x^2+y^2+z^2 < min(t, 1-t)^2.  The first n
         * accepted candidates, in candidate order, are kept. */
        uint64_t s = or_stream_key(seed, 1);
        int64_t got = 0;
        for (uint64_t c = 0; got < n; c++) {
            uint64_t kt = or_output(s, 4 * c) >> 11;
            double t = (double)kt * 0x1.0p-53;
            double x = or_unit(or_output(s, 4 * c + 1)) - 0.5;
            double y = or_unit(or_output(s, 4 * c + 2)) - 0.5;
            double z = or_unit(or_output(s, 4 * c + 3)) - 0.5;
            double r = t < 1.0 - t ? t : 1.0 - t;
            double rr = x * x + y * y;
            rr = rr + z * z;
            if (rr < r * r) {
                raw[0 * n + got] = t;
                raw[1 * n + got] = x;
                raw[2 * n + got] = y;
                raw[3 * n + got] = z;
                keys[got].key = kt;
                keys[got].gen = got;
                got++;
            }
        }
    } else if (region == OR_MINK3_DIAMOND) {
        /* 2+1 Alexandrov interval of height 1 between (0,0,0) and (1,0,0): candidates
         * uniform in [0,1) x [-1/2,1/2)^2, accepted when x^2+y^2 < min(t, 1-t)^2; the
         * first n accepted, in candidate order, are kept (acceptance pi/12). */
        uint64_t s = or_stream_key(seed, 5);
        int64_t got = 0;
        for (uint64_t c = 0; got < n; c++) {
            uint64_t kt = or_output(s, 3 * c) >> 11;
            double t = (double)kt * 0x1.0p-53;
            double x = or_unit(or_output(s, 3 * c + 1)) - 0.5;
            double y = or_unit(or_output(s, 3 * c + 2)) - 0.5;
            double r = t < 1.0 - t ? t : 1.0 - t;
            double rr = x * x + y * y;
            if (rr < r * r) {
                raw[0 * n + got] = t;
                raw[1 * n + got] = x;
                raw[2 * n + got] = y;
                keys[got].key = kt;
                keys[got].gen = got;
                got++;
            }
        }
    } else if (region == OR_DS2_SLAB) {
        /* 1+1 de Sitter slab, spherical foliation, eta in [-eta0, eta0], theta on
         * the circle.  The conformal-time density is proportional to sec^2(eta) =
         * d tan(eta) / d eta, so x = tan(eta) is uniform on [-tan eta0, tan eta0]
         * (computed exactly up to one rounding); eta = atan(x); theta = 2 pi w.
         * Time order by x, which is monotone in eta. */
        double X = tan(eta0);
        double two_pi = 2.0 * M_PI;
        uint64_t s = or_stream_key(seed, 4);
        for (int64_t g = 0; g < n; g++) {
            double u = or_unit(or_output(s, 2 * (uint64_t)g));
            double w = or_unit(or_output(s, 2 * (uint64_t)g + 1));
            double x = (2.0 * u - 1.0) * X;
            raw[0 * n + g] = x;
            raw[1 * n + g] = atan(x);
            raw[2 * n + g] = two_pi * w;
            keys[g].key = or_order_bits(x);
            keys[g].gen = g;
        }
    } else {
        /* 3+1 de Sitter slab, spherical foliation, eta in [-eta0, eta0]:
         * the conformal-time density is proportional to sec^4(eta).  With
         * x = tan(eta), sec^4(eta) d(eta) = (1 + x^2) dx, so the CDF is linear
         * in x + x^3/3 and the inverse is the real root of the cubic
         * x^3 + 3x - 3y = 0:  x = 2 sinh(asinh(3y/2)/3).
         * The S^3 direction is a cube-rejected point of B^4, normalised. */
        double X = tan(eta0);
        double Y = X + ((X * X) * X) / 3.0;
        uint64_t sx = or_stream_key(seed, 2);
        uint64_t sn = or_stream_key(seed, 3);
        for (int64_t g = 0; g < n; g++) {
            double u = or_unit(or_output(sx, (uint64_t)g));
            double y = (2.0 * u - 1.0) * Y;
            double x = 2.0 * sinh(asinh(1.5 * y) / 3.0);
            double c = 1.0 / sqrt(1.0 + x * x);
            double sn_eta = x * c;
            uint64_t ps = or_output(sn, (uint64_t)g);  /* per-point generator state */
            /* Try k draws 4k..4k+3 as a point of [-1,1)^4; keep the first one inside
             * the unit ball (and not at its centre).  After 4096 failures (probability
             * 0.69^4096) the direction (1,0,0,0) is used so the loop is bounded. */
            double a[4] = {1.0, 0.0, 0.0, 0.0}, r2 = 1.0;
            for (uint64_t k = 0; k < 4096; k++) {
                double b[4];
                for (int q = 0; q < 4; q++)
                    b[q] = 2.0 * or_unit(or_output(ps, 4 * k + (uint64_t)q)) - 1.0;
                double s2 = b[0] * b[0] + b[1] * b[1];
                s2 = s2 + b[2] * b[2];
                s2 = s2 + b[3] * b[3];
                if (s2 < 1.0 && s2 > 0x1.0p-40) {
                    for (int q = 0; q < 4; q++) a[q] = b[q];
                    r2 = s2;
                    break;
                }
            }
            double r = sqrt(r2);
            raw[0 * n + g] = x;
            raw[1 * n + g] = c;
            raw[2 * n + g] = sn_eta;
            for (int q = 0; q < 4; q++) raw[(3 + q) * n + g] = a[q] / r;
            keys[g].key = or_order_bits(x);
            keys[g].gen = g;
        }
    }

    qsort(keys, (size_t)n, sizeof(or_sortkey), or_cmp_key);
    for (int64_t i = 0; i < n; i++)
        for (int p = 0; p < planes; p++)
            coords[(int64_t)p * n + i] = raw[(int64_t)p * n + keys[i].gen];
    free(raw);
    free(keys);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Causal relation (strict: null and equal-time pairs are unrelated)          */
/* ------------------------------------------------------------------------- */

/* Is i ≺ j?  Only asked with i < j in time order. */
static int or_related(int region, const double *c, int64_t n, int64_t i, int64_t j)
{
    if (region == OR_MINK2_DIAMOND) {
        return c[i] < c[j] && c[n + i] < c[n + j];
    } else if (region == OR_MINK4_DIAMOND) {
        double dt = c[j] - c[i];
        if (!(dt > 0.0)) return 0;
        double dx = c[n + j] - c[n + i];
        double dy = c[2 * n + j] - c[2 * n + i];
        double dz = c[3 * n + j] - c[3 * n + i];
        double s = dx * dx + dy * dy;
        s = s + dz * dz;
        return dt * dt > s;
    } else if (region == OR_MINK3_DIAMOND) {
        double dt = c[j] - c[i];
        if (!(dt > 0.0)) return 0;
        double dx = c[n + j] - c[n + i];
        double dy = c[2 * n + j] - c[2 * n + i];
        return dt * dt > dx * dx + dy * dy;
    } else if (region == OR_DS2_SLAB) {
        /* Timelike on the cylinder: the angular separation, measured the short way
         * round, pi - |pi - |theta_i - theta_j||, is below the conformal-time
         * separation eta_j - eta_i (strict on both counts). */
        double deta = c[n + j] - c[n + i];
        if (!(c[n + i] < c[n + j])) return 0;
        double dth = fabs(c[2 * n + i] - c[2 * n + j]);
        dth = M_PI - fabs(M_PI - dth);
        return dth < deta;
    } else {
        /* Delta eta > great-circle angle  <=>  cos(Delta eta) < n_i . n_j, valid
         * because both angles lie in [0, pi] (Delta eta <= 2 eta0 < pi). */
        if (!(c[i] < c[j])) return 0;
        double cdeta = c[n + i] * c[n + j] + c[2 * n + i] * c[2 * n + j];
        double dot = c[3 * n + i] * c[3 * n + j] + c[4 * n + i] * c[4 * n + j];
        dot = dot + c[5 * n + i] * c[5 * n + j];
        dot = dot + c[6 * n + i] * c[6 * n + j];
        return cdeta < dot;
    }
}

int64_t or_ld_words(int64_t n) { return ((n + 511) / 512) * 8; }

/* Symmetric causal matrix S = C + C^T as packed rows: bit j of row i is
 * bit (j & 63) of word i*ld + (j >> 6).  Row by row, each pair tested with the
 * earlier element first, so every row is written by exactly one thread. */
int or_causal_matrix(int region, const double *coords, int64_t n, uint64_t *bits, int64_t ld)
{
    if (or_coord_planes(region) < 0 || n < 1 || ld * 64 < n) return -1;
    memset(bits, 0, sizeof(uint64_t) * (size_t)n * (size_t)ld);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        uint64_t *row = bits + i * ld;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            int r = i < j ? or_related(region, coords, n, i, j)
                          : or_related(region, coords, n, j, i);
            if (r) row[j >> 6] |= 1ULL << (j & 63);
        }
    }
    return 0;
}

/* Selected rows of the same matrix: out[r*ld ...] is row rows[r]. */
int or_causal_rows(int region, const double *coords, int64_t n, const int64_t *rows,
                   int64_t nrows, uint64_t *out, int64_t ld)
{
    if (or_coord_planes(region) < 0 || n < 1 || ld * 64 < n) return -1;
    memset(out, 0, sizeof(uint64_t) * (size_t)nrows * (size_t)ld);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; r++) {
        int64_t i = rows[r];
        uint64_t *row = out + r * ld;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            int rel = i < j ? or_related(region, coords, n, i, j)
                            : or_related(region, coords, n, j, i);
            if (rel) row[j >> 6] |= 1ULL << (j & 63);
        }
    }
    return 0;
}

static int or_bit(const uint64_t *bits, int64_t ld, int64_t i, int64_t j)
{
    return (int)((bits[i * ld + (j >> 6)] >> (j & 63)) & 1ULL);
}

/* ------------------------------------------------------------------------- */
/* Interval abundances                                                         */
/* ------------------------------------------------------------------------- */

/* Definitional tier, from the inclusive order intervals (eq. IOIs) and the Alexandroff
 * set A_ij = J+(i) ∩ J-(j) of Sec. 2 (set algorithms): for every element j and every i in
 * its past J-(j), the size of A_ij is the number of k in J-(j) that also lie in J+(i);
 * the pair then belongs to L_{|A_ij|+1}(j), so N_m = sum_j |L_{m+1}(j)| counts the related
 * pairs with m elements inside.  This is the quantity the naive algorithm of Sec. 4.2
 * computes, but organised around each element's past as the interval definition is.
 * Only labels below j can precede j (time order), and elements k of A_ij lie strictly
 * between i and j.  One private histogram per thread, summed at the end.  hist has n-1
 * bins (counts 0..n-2; the thesis's n_m is hist[m-1]). */
static void or_past_intervals(const uint64_t *bits, int64_t ld, int64_t j, uint64_t *mine)
{
    for (int64_t i = 0; i < j; i++) {
        if (!or_bit(bits, ld, j, i)) continue;        /* i in J-(j) */
        int64_t size = 0;
        for (int64_t k = i + 1; k < j; k++)
            if (or_bit(bits, ld, j, k) && or_bit(bits, ld, i, k)) size++;  /* k in J-(j), J+(i) */
        mine[size]++;
    }
}

int or_histogram_naive(const uint64_t *bits, int64_t n, int64_t ld, uint64_t *hist)
{
    if (n < 2) return -1;
    int64_t nb = n - 1;
    memset(hist, 0, sizeof(uint64_t) * (size_t)nb);
#pragma omp parallel
    {
        uint64_t *mine = (uint64_t *)calloc((size_t)nb, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 1)
        for (int64_t j = n - 1; j >= 1; j--) or_past_intervals(bits, ld, j, mine);
#pragma omp critical
        for (int64_t m = 0; m < nb; m++) hist[m] += mine[m];
        free(mine);
    }
    return 0;
}

/* The definitional tier over a list of elements j only (every i in J-(j)): a bounded
 * sample of the full count, used to time the CPU. */
int or_histogram_naive_elems(const uint64_t *bits, int64_t n, int64_t ld, uint64_t *hist,
                             const int64_t *elems, int64_t nelems)
{
    if (n < 2) return -1;
    int64_t nb = n - 1;
    for (int64_t e = 0; e < nelems; e++)
        if (elems[e] < 0 || elems[e] >= n) return -1;
    memset(hist, 0, sizeof(uint64_t) * (size_t)nb);
#pragma omp parallel
    {
        uint64_t *mine = (uint64_t *)calloc((size_t)nb, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 1)
        for (int64_t e = 0; e < nelems; e++) or_past_intervals(bits, ld, elems[e], mine);
#pragma omp critical
        for (int64_t m = 0; m < nb; m++) hist[m] += mine[m];
        free(mine);
    }
    return 0;
}

/* Interval size of one pair by word AND + popcount over columns (i, j). */
int64_t or_pair_interval(const uint64_t *bits, int64_t ld, int64_t i, int64_t j)
{
    int64_t lo = i + 1, hi = j; /* columns [lo, hi) */
    if (lo >= hi) return 0;
    const uint64_t *a = bits + i * ld, *b = bits + j * ld;
    int64_t w0 = lo >> 6, w1 = (hi - 1) >> 6;
    int64_t x = 0;
    for (int64_t w = w0; w <= w1; w++) {
        uint64_t m = ~0ULL;
        if (w == w0) m &= ~0ULL << (lo & 63);
        if (w == w1) m &= ~0ULL >> (63 - ((hi - 1) & 63));
        x += __builtin_popcountll(a[w] & b[w] & m);
    }
    return x;
}

/* Alg. "Optimized Interval Abundance Measurement" on the CPU, restricted to
 * rows i in [row_begin, row_end) (the full histogram for 0..n-1).  Private
 * per-thread histograms are summed at the end. Returns the pairs counted. */
int64_t or_histogram_fast(const uint64_t *bits, int64_t n, int64_t ld, uint64_t *hist,
                          int64_t row_begin, int64_t row_end)
{
    if (n < 2 || row_begin < 0 || row_end > n || row_begin > row_end) return -1;
    int64_t nb = n - 1, pairs = 0;
    memset(hist, 0, sizeof(uint64_t) * (size_t)nb);
#pragma omp parallel reduction(+ : pairs)
    {
        uint64_t *mine = (uint64_t *)calloc((size_t)nb, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = row_begin; i < row_end; i++) {
            for (int64_t j = i + 1; j < n; j++) {
                if (!or_bit(bits, ld, i, j)) continue;
                mine[or_pair_interval(bits, ld, i, j)]++;
                pairs++;
            }
        }
#pragma omp critical
        for (int64_t m = 0; m < nb; m++) hist[m] += mine[m];
        free(mine);
    }
    return pairs;
}

/* The same tier over an arbitrary list of rows i (all j > i): a bounded sample of
 * the full count, used to time the CPU.  Returns the pairs counted. */
int64_t or_histogram_fast_rows(const uint64_t *bits, int64_t n, int64_t ld, uint64_t *hist,
                               const int64_t *rows, int64_t nrows)
{
    if (n < 2) return -1;
    int64_t nb = n - 1, pairs = 0;
    memset(hist, 0, sizeof(uint64_t) * (size_t)nb);
#pragma omp parallel reduction(+ : pairs)
    {
        uint64_t *mine = (uint64_t *)calloc((size_t)nb, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < nrows; r++) {
            int64_t i = rows[r];
            for (int64_t j = i + 1; j < n; j++) {
                if (!or_bit(bits, ld, i, j)) continue;
                mine[or_pair_interval(bits, ld, i, j)]++;
                pairs++;
            }
        }
#pragma omp critical
        for (int64_t m = 0; m < nb; m++) hist[m] += mine[m];
        free(mine);
    }
    return pairs;
}

/* In- and out-degrees (past and future set sizes) of every element and the
 * number of 3-chains i ≺ k ≺ j, which equals sum_n n*N_n. */
int or_degrees(const uint64_t *bits, int64_t n, int64_t ld, int64_t *indeg, int64_t *outdeg,
               uint64_t *chains3, uint64_t *relations)
{
    uint64_t c3 = 0, rel = 0;
#pragma omp parallel for reduction(+ : c3, rel) schedule(static)
    for (int64_t i = 0; i < n; i++) {
        int64_t in = 0, out = 0;
        for (int64_t j = 0; j < n; j++) {
            if (!or_bit(bits, ld, i, j)) continue;
            if (j < i) in++; else out++;
        }
        indeg[i] = in;
        outdeg[i] = out;
        c3 += (uint64_t)in * (uint64_t)out;
        rel += (uint64_t)out;
    }
    *chains3 = c3;
    *relations = rel;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Benincasa-Dowker action in quadruple precision                              */
/* ------------------------------------------------------------------------- */
typedef __float128 q_t;

static q_t q_sqrt(q_t a)   /* Newton from the double root; two steps reach quad */
{
    if (a <= 0) return 0;
    q_t r = (q_t)sqrt((double)a);
    r = (r + a / r) / 2;
    r = (r + a / r) / 2;
    r = (r + a / r) / 2;
    return r;
}

static q_t q_powi(q_t b, int64_t e)  /* b^e, e >= 0, with 0^0 = 1 */
{
    q_t r = 1;
    while (e > 0) {
        if (e & 1) r *= b;
        b *= b;
        e >>= 1;
    }
    return r;
}

/* Smearing functions written as sum_k c_k(n) eps^k (1-eps)^(n-k), k <= min(n, K):
 * the thesis's f_d(n, eps) multiplied out, so no power of (1-eps) is negative
 * and eps = 1 is allowed (then f reduces to the local coefficients).
 *   f_2: c_0 = 1, c_1 = -2n, c_2 = n(n-1)/2
 *   f_4: c_0 = 1, c_1 = -9n, c_2 = 8n(n-1), c_3 = -(4/3) n(n-1)(n-2) */
static q_t or_smear(int dim, int64_t n, q_t eps)
{
    q_t nn = (q_t)n, c[4];
    int K;
    if (dim == 2) {
        c[0] = 1; c[1] = -2 * nn; c[2] = nn * (nn - 1) / 2; K = 2;
    } else if (dim == 3) {
        c[0] = 1; c[1] = -(q_t)27 / 8 * nn; c[2] = (q_t)9 / 8 * nn * (nn - 1); K = 2;
    } else {
        c[0] = 1; c[1] = -9 * nn; c[2] = 8 * nn * (nn - 1);
        c[3] = -(q_t)4 * nn * (nn - 1) * (nn - 2) / 3; K = 3;
    }
    q_t f = 0, om = 1 - eps;
    for (int k = 0; k <= K && k <= n; k++)
        f += c[k] * q_powi(eps, k) * q_powi(om, n - k);
    return f;
}

/* The 2+1 prefactor (1 / Gamma(5/3)) (pi / (3 sqrt 2))^(2/3) (eq. s3d_local, l = l_p). */
static q_t or_c3(void)
{
    q_t p = M_PIq / (3 * sqrtq(2));
    return cbrtq(p * p) / tgammaq((q_t)5 / 3);
}

/*
 * Action from the abundances hist[0..n-2] (hist[m] = N_m, pairs with m elements
 * inside).  dim 2, 3 or 4.  eps == 0 selects the local action:
 *   S^(1+1) = 2 (N - 2N_0 + 4N_1 - 2N_2)
 *   S^(2+1) = C_3 (N - N_0 + (27/8) N_1 - (9/4) N_2)
 *   S^(3+1) = (4/sqrt 6) (N - N_0 + 9N_1 - 16N_2 + 8N_3)        (l = l_p)
 * with C_3 = (pi / (3 sqrt 2))^(2/3) / Gamma(5/3).  0 < eps <= 1 selects the smeared action:
 *   S_eps^(1+1) = 2 eps [N - 2 eps sum_m N_m f_2(m, eps)]
 *   S_eps^(2+1) = C_3 eps^(2/3) [N - eps sum_m N_m f_3(m, eps)]
 *   S_eps^(3+1) = 4 sqrt(eps/6) [N - eps sum_m N_m f_4(m, eps)]
 * Out: *out = S rounded once to double; *kappa = (N + eps_c sum|N_m f_m|)/|bracket|
 * (1 for the local action).  Returns 0, or -1 on bad arguments.
 */
int or_action(const uint64_t *hist, int64_t n, int dim, double eps, double *out, double *kappa)
{
    if (n < 2 || (dim != 2 && dim != 3 && dim != 4) || eps < 0.0 || eps > 1.0) return -1;
    int64_t nb = n - 1;
    if (eps == 0.0) {
        int64_t h[4] = {0, 0, 0, 0};
        for (int m = 0; m < 4 && m < nb; m++) h[m] = (int64_t)hist[m];
        q_t s;
        if (dim == 2) {
            int64_t I = n - 2 * h[0] + 4 * h[1] - 2 * h[2];
            s = 2 * (q_t)I;
        } else if (dim == 3) {
            int64_t I8 = 8 * n - 8 * h[0] + 27 * h[1] - 18 * h[2];  /* 8 times the bracket */
            s = or_c3() * (q_t)I8 / 8;
        } else {
            int64_t I = n - h[0] + 9 * h[1] - 16 * h[2] + 8 * h[3];
            s = 4 / q_sqrt(6) * (q_t)I;
        }
        *out = (double)s;
        if (kappa) *kappa = 1.0;
        return 0;
    }
    q_t e = (q_t)eps, sum = 0, asum = 0;
    for (int64_t m = 0; m < nb; m++) {
        if (!hist[m]) continue;
        q_t t = (q_t)hist[m] * or_smear(dim, m, e);
        sum += t;
        asum += t < 0 ? -t : t;
    }
    q_t ec = dim == 2 ? 2 * e : e;
    q_t bracket = (q_t)n - ec * sum;
    q_t pref = dim == 2 ? 2 * e : dim == 3 ? or_c3() * cbrtq(e * e) : 4 * q_sqrt(e / 6);
    *out = (double)(pref * bracket);
    if (kappa) {
        q_t ab = bracket < 0 ? -bracket : bracket;
        *kappa = ab > 0 ? (double)(((q_t)n + ec * asum) / ab) : INFINITY;
    }
    return 0;
}

/* The smearing weight itself, rounded to double (for tests). */
double or_smear_weight(int dim, int64_t m, double eps)
{
    return (double)or_smear(dim, m, (q_t)eps);
}

int or_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------- */
/* Discrete d'Alembertian (Sec. 4.1, eqs. b2d_local and b4d_local)            */
/* ------------------------------------------------------------------------- */

/*
 * B phi(j) = (K / ell^2) [ -phi(j) + sum_m c_m sum_{i in L_m(j)} phi(i) ] for every j,
 * with L_m(j) = { i ≺ j : exactly m-1 elements strictly between i and j }:
 *   1+1: K = 2,          c = ( 2, -4,  2)      (the bracket 2 (L1 - 2 L2 + L3))
 *   2+1: K = C_3,        c = ( 1, -27/8, 9/4)   (eq. b3d_local, C_3 as for the action)
 *   3+1: K = 4/sqrt(6),  c = ( 1, -9, 16, -8)
 * Sums and constants in __float128, one rounding at the end.  Optional outputs for
 * error bounds of other summation orders: terms[j] = 1 + |L_1(j)| + ... (the number
 * of summands) and abs_sum[j] = |phi(j)| + sum_m |c_m| sum_{i in L_m(j)} |phi(i)|.
 * Returns 0, or -1 on bad arguments.
 */
static int or_dal_run(const uint64_t *bits, int64_t n, int64_t ld, int dim, double ell,
                      const double *phi, const int64_t *js, int64_t count, double *out,
                      int64_t *terms, double *abs_sum)
{
    q_t K;
    int layers;
    q_t c[4];
    if (dim == 2) {
        K = 2; layers = 3; c[0] = 2; c[1] = -4; c[2] = 2; c[3] = 0;
    } else if (dim == 3) {
        K = or_c3(); layers = 3; c[0] = 1; c[1] = -(q_t)27 / 8; c[2] = (q_t)9 / 4; c[3] = 0;
    } else if (dim == 4) {
        K = 4 / q_sqrt(6); layers = 4; c[0] = 1; c[1] = -9; c[2] = 16; c[3] = -8;
    } else {
        return -1;
    }
    if (n < 1 || ld * 64 < n || !(ell > 0.0)) return -1;
    const q_t scale = K / ((q_t)ell * (q_t)ell);
    for (int64_t x = 0; x < count; x++)
        if (js && (js[x] < 0 || js[x] >= n)) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t x = 0; x < count; x++) {
        const int64_t j = js ? js[x] : x;
        q_t sum = -(q_t)phi[j], mag = fabs(phi[j]);
        int64_t cnt = 1;
        for (int64_t i = 0; i < j; i++) {
            if (!or_bit(bits, ld, j, i)) continue;      /* i ≺ j (i earlier) */
            int64_t m = or_pair_interval(bits, ld, i, j); /* |L| index m+1 */
            if (m >= layers) continue;
            sum += c[m] * (q_t)phi[i];
            mag += fabs((double)c[m]) * fabs(phi[i]);
            cnt++;
        }
        out[x] = (double)(scale * sum);
        if (terms) terms[x] = cnt;
        if (abs_sum) abs_sum[x] = (double)mag;
    }
    return 0;
}

int or_dalembertian(const uint64_t *bits, int64_t n, int64_t ld, int dim, double ell,
                    const double *phi, double *out, int64_t *terms, double *abs_sum)
{
    return or_dal_run(bits, n, ld, dim, ell, phi, NULL, n, out, terms, abs_sum);
}

/* The same for the elements js[0 .. count-1] only (outputs in list order). */
int or_dalembertian_cols(const uint64_t *bits, int64_t n, int64_t ld, int dim, double ell,
                         const double *phi, const int64_t *js, int64_t count, double *out,
                         int64_t *terms, double *abs_sum)
{
    if (!js || count < 0) return -1;
    return or_dal_run(bits, n, ld, dim, ell, phi, js, count, out, terms, abs_sum);
}

/* The 2+1 prefactor rounded to double (for tests). */
double or_c3_double(void) { return (double)or_c3(); }

/* ------------------------------------------------------------------------- */
/* Longest chains inside Alexandroff sets (Sec. 2.5.2 "Set Partitions",        */
/* algorithm "Maximal Chain Length").                                          */
/*                                                                             */
/* Indices -1 and n name two virtual elements, one below and one above every  */
/* element.  A chain's length is its number of links (relations between       */
/* consecutive elements), which is what the algorithm returns.  Labels are a  */
/* linear extension of the order, so a ≺ m ≺ b forces a < m < b.              */
/* ------------------------------------------------------------------------- */

/* Word w of the Alexandroff set A_ab = {m : a ≺ m ≺ b}. */
static uint64_t or_between_word(const uint64_t *bits, int64_t ld, int64_t n, int64_t a,
                                int64_t b, int64_t w)
{
    const int64_t lo = a + 1 > 0 ? a + 1 : 0, hi = b < n ? b : n; /* indices [lo, hi) */
    const int64_t base = w << 6;
    if (base + 64 <= lo || base >= hi) return 0;
    uint64_t m = ~0ULL;
    if (lo > base) m &= ~0ULL << (lo - base);
    if (hi < base + 64) m &= ~0ULL >> (base + 64 - hi);
    if (a >= 0) m &= bits[a * ld + w]; /* a ≺ m (m later than a and related) */
    if (b < n) m &= bits[b * ld + w];  /* m ≺ b */
    return m;
}

/* Links on the longest chain from k to j: the recursion of the algorithm.  For
 * every element m of A_kj the distance from m to j is taken from dist[] when known
 * (-1 marks "not yet"), else computed by the same recursion on A_mj and stored; an
 * element whose own Alexandroff set with j is empty is one link from j.  The result
 * is one link more than the largest of those distances (one link when A_kj is empty).
 * dist[] belongs to this j only. */
static int64_t or_chain_down(const uint64_t *bits, int64_t ld, int64_t n, int64_t k, int64_t j,
                             int64_t *dist)
{
    int64_t best = 0;
    const int64_t first = k + 1 > 0 ? k + 1 : 0, last = (j < n ? j : n) - 1;
    for (int64_t w = first >> 6; first <= last && w <= last >> 6; w++) {
        uint64_t x = or_between_word(bits, ld, n, k, j, w);
        while (x) { /* scan the set bits one by one (Alg. "Non-Zero Elements") */
            const int64_t m = (w << 6) + __builtin_ctzll(x);
            x &= x - 1;
            if (dist[m] < 0) dist[m] = or_chain_down(bits, ld, n, m, j, dist);
            if (dist[m] > best) best = dist[m];
        }
    }
    return best + 1;
}

/* The same recursion entered from the past end: links on the longest chain from i up to
 * k, with dist[m] caching the distance from i to m (this i only). */
static int64_t or_chain_up(const uint64_t *bits, int64_t ld, int64_t n, int64_t i, int64_t k,
                           int64_t *dist)
{
    int64_t best = 0;
    const int64_t first = i + 1 > 0 ? i + 1 : 0, last = (k < n ? k : n) - 1;
    for (int64_t w = first >> 6; first <= last && w <= last >> 6; w++) {
        uint64_t x = or_between_word(bits, ld, n, i, k, w);
        while (x) {
            const int64_t m = (w << 6) + __builtin_ctzll(x);
            x &= x - 1;
            if (dist[m] < 0) dist[m] = or_chain_up(bits, ld, n, i, m, dist);
            if (dist[m] > best) best = dist[m];
        }
    }
    return best + 1;
}

/* a ≺ b, for real or virtual a < b. */
static int or_precedes(const uint64_t *bits, int64_t ld, int64_t n, int64_t a, int64_t b)
{
    if (a < 0 || b >= n) return 1;
    return or_bit(bits, ld, a, b);
}

/*
 * For each pair s, with -1 <= lo[s] < hi[s] <= n:
 *   length[s]        links on the longest chain from lo[s] to hi[s]; 0 when lo[s] does
 *                    not precede hi[s];
 *   height[s*n + k]  (when height is not NULL) links on the longest chain from lo[s] to k,
 *                    for every k with lo[s] ≺ k and (k ≺ hi[s] or k = hi[s]); 0 elsewhere.
 * Returns 0, or -1 on bad arguments.
 */
int or_longest_chain(const uint64_t *bits, int64_t n, int64_t ld, const int64_t *lo,
                     const int64_t *hi, int64_t count, int64_t *length, int64_t *height)
{
    if (n < 1 || ld * 64 < n || count < 0) return -1;
    for (int64_t s = 0; s < count; s++)
        if (lo[s] < -1 || hi[s] > n || lo[s] >= hi[s] || lo[s] >= n || hi[s] < 0) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < count; s++) {
        const int64_t a = lo[s], b = hi[s];
        int64_t *dist = (int64_t *)malloc((size_t)n * sizeof(int64_t));
        const int related = or_precedes(bits, ld, n, a, b);
        for (int64_t m = 0; m < n; m++) dist[m] = -1;
        length[s] = related ? or_chain_down(bits, ld, n, a, b, dist) : 0;
        if (height) {
            int64_t *h = height + s * n;
            for (int64_t m = 0; m < n; m++) { h[m] = 0; dist[m] = -1; }
            if (related) {
                /* latest first, so that the recursion (not the loop order) fills dist[] */
                const int64_t top = b < n ? b : n - 1, first = a + 1 > 0 ? a + 1 : 0;
                for (int64_t k = top; k >= first; k--) {
                    const int in = or_precedes(bits, ld, n, a, k) &&
                                   (k == b || or_precedes(bits, ld, n, k, b));
                    if (!in) continue;
                    if (dist[k] < 0) dist[k] = or_chain_up(bits, ld, n, a, k, dist);
                    h[k] = dist[k];
                }
            }
        }
        free(dist);
    }
    return 0;
}
