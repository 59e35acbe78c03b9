/*
 * fisher_oracle.c -- plain CPU oracle for the Monte-Carlo Fisher exact test
 * consumer of the streams (Section 4 of the clrng paper).
 *
 * TEST INFRASTRUCTURE ONLY (see mrg_oracle.c); shares nothing with the GPU
 * path.
 *
 * Section 4: for each replicate, a random table with the observed margins is
 * sampled cell by cell, row by row, each entry drawn by inversion of its
 * conditional distribution given the entries already drawn, with one U(0,1)
 * number; (I-1)(J-1) numbers per table, the last row and column being
 * determined.  The statistic of a table is -sum log(n_ij!); the count is the
 * number of replicates whose statistic is at most the observed one; the
 * p-value is (1 + count) / (B + 1).
 *
 * Reading (the paper says "standard inversion"): entry (i, j) given the
 * entries before it is hypergeometric: from the N' units still unassigned in
 * columns j..J-1 of rows i..I-1, of which K = remaining total of column j are
 * in column j, row i takes n = its remaining total.  Its pmf over
 * x in [lo, hi], lo = max(0, n - (N' - K)), hi = min(n, K), is proportional to
 * weights with w(lo) = 1 and
 *     w(x+1) = w(x) * ((K - x) (n - x)) / ((x + 1) (N' - K - n + x + 1)),
 * evaluated in double precision in this order (products exact, one rounded
 * multiply, one rounded divide).  The entry is the smallest x with
 * u * W <= w(lo) + ... + w(x), W = w(lo) + ... + w(hi), sums taken in order.
 * Built with -ffp-contract=off.
 *
 * The weights can exceed the double range: w(mode)/w(lo) = pmf(mode)/pmf(lo)
 * passes 2^1024 for some entries of the day-of-week table of Section 4.2.
 * They are therefore carried with an extended exponent: whenever a weight
 * exceeds 2^600, it and the running sum are multiplied by 2^-600 (exact), and
 * the search compares u * W with the running sum brought to W's scale.  Every
 * mantissa is the one of the same double-precision operations on an unbounded
 * exponent range, so nothing changes where nothing overflowed.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

uint64_t orc_step(int gen, uint32_t state[6]);
double orc_norm(int gen);

enum { FT_MAX = 5, FT_DIM = 32 };

#define ORC_BIG 0x1p600
#define ORC_SCALE_EXP 600

/* One entry by inversion of its conditional distribution. */
int orc_hyper_invert(double u, int64_t Np, int64_t K, int64_t n) {
    int64_t lo = n - (Np - K);
    if (lo < 0) lo = 0;
    int64_t hi = n < K ? n : K;
    if (hi <= lo) return (int)lo;
    /* W = w(lo) + ... + w(hi); `scales` counts the 2^-600 rescalings */
    double W = 0.0, w = 1.0;
    int scales = 0;
    for (int64_t x = lo; x <= hi; ++x) {
        W += w;
        if (x < hi) {
            double num = (double)((K - x) * (n - x));
            double den = (double)((x + 1) * (Np - K - n + x + 1));
            w = w * num / den;
            if (w > ORC_BIG) {
                w = ldexp(w, -ORC_SCALE_EXP);
                W = ldexp(W, -ORC_SCALE_EXP);
                ++scales;
            }
        }
    }
    double target = u * W;
    /* the same running sums again, each compared at W's scale */
    double s = 0.0;
    w = 1.0;
    int done = 0;
    for (int64_t x = lo; x <= hi; ++x) {
        s += w;
        if (target <= ldexp(s, -ORC_SCALE_EXP * (scales - done))) return (int)x;
        double num = (double)((K - x) * (n - x));
        double den = (double)((x + 1) * (Np - K - n + x + 1));
        w = w * num / den;
        if (w > ORC_BIG) {
            w = ldexp(w, -ORC_SCALE_EXP);
            s = ldexp(s, -ORC_SCALE_EXP);
            ++done;
        }
    }
    return (int)hi;
}

/* Sample one I x J table (I, J <= 32) into tab[i * ld + j] with row totals
 * r[] and column totals c[] from the 6-word stream state, which advances
 * (I-1)(J-1) steps.  Returns 0, or -1 when the margins disagree. */
int orc_table_sample_ld(int gen, uint32_t state[6], int I, int J, const int32_t* r, const int32_t* c,
                        int32_t* tab, int ld) {
    int64_t crem[FT_DIM];
    int64_t rsum = 0, csum = 0;
    if (I < 1 || J < 1 || I > FT_DIM || J > FT_DIM) return -1;
    for (int i = 0; i < I; ++i) rsum += r[i];
    for (int j = 0; j < J; ++j) {
        crem[j] = c[j];
        csum += c[j];
    }
    if (rsum != csum) return -1;
    double norm = orc_norm(gen);
    for (int i = 0; i < I - 1; ++i) {
        int64_t rrem = r[i];
        int64_t Np = 0;  /* units left in columns j..J-1 over rows i..I-1 */
        for (int j = 0; j < J; ++j) Np += crem[j];
        for (int j = 0; j < J - 1; ++j) {
            double u = (double)orc_step(gen, state) * norm;
            int x = orc_hyper_invert(u, Np, crem[j], rrem);
            tab[i * ld + j] = x;
            rrem -= x;
            Np -= crem[j];
            crem[j] -= x;
        }
        tab[i * ld + J - 1] = (int32_t)rrem;
        crem[J - 1] -= rrem;
    }
    for (int j = 0; j < J; ++j) tab[(I - 1) * ld + j] = (int32_t)crem[j];
    return 0;
}

/* -sum log(n_ij!) over the I x J cells of tab[i * ld + j], row-major, each
 * log(n!) = lgamma(n + 1) evaluated in long double and rounded to double,
 * the sum taken in double. */
double orc_table_stat_ld(int I, int J, const int32_t* tab, int ld) {
    double s = 0.0;
    for (int i = 0; i < I; ++i)
        for (int j = 0; j < J; ++j) s -= (double)lgammal((long double)tab[i * ld + j] + 1.0L);
    return s;
}

/* Tables t = 0..n-1 from streams t (18-word records, current state advanced
 * in place): shapes I[t] x J[t] (<= 5 x 5), margins rows[t][5], cols[t][5];
 * outputs tabs[t][5][5] (zero padded) and stats[t] (may be NULL). */
int orc_tables(int gen, uint32_t* streams, uint64_t n, const int32_t* I, const int32_t* J,
               const int32_t* rows, const int32_t* cols, int32_t* tabs, double* stats) {
    for (uint64_t t = 0; t < n; ++t) {
        int32_t* tab = tabs + t * FT_MAX * FT_MAX;
        memset(tab, 0, FT_MAX * FT_MAX * sizeof(int32_t));
        if (I[t] > FT_MAX || J[t] > FT_MAX) return -1;
        int rc = orc_table_sample_ld(gen, streams + t * 18, I[t], J[t], rows + t * FT_MAX, cols + t * FT_MAX,
                                     tab, FT_MAX);
        if (rc) return rc;
        if (stats) stats[t] = orc_table_stat_ld(I[t], J[t], tab, FT_MAX);
    }
    return 0;
}

/* Section 4: B replicates of the observed I x J table (row-major, stride J),
 * replicate b from stream b.  Returns the number of replicates whose
 * statistic is at most the observed one; *observed_stat receives that.
 * Reading: "at most" with R's near-tie rule, statistic <= observed /
 * (1 + 64 eps), so that tables whose statistic equals the observed one
 * mathematically count whatever the last bit of their rounded sums (Section 4
 * compares with stats::fisher.test, which counts this way). */
uint64_t orc_fisher_count(int gen, uint32_t* streams, uint64_t B, int I, int J, const int32_t* observed,
                          double* observed_stat) {
    int32_t r[FT_DIM] = {0}, c[FT_DIM] = {0}, tab[FT_DIM * FT_DIM];
    for (int i = 0; i < I; ++i)
        for (int j = 0; j < J; ++j) {
            r[i] += observed[i * J + j];
            c[j] += observed[i * J + j];
        }
    double o = orc_table_stat_ld(I, J, observed, J);
    if (observed_stat) *observed_stat = o;
    const double threshold = o / (1.0 + 64.0 * DBL_EPSILON);
    uint64_t count = 0;
    for (uint64_t b = 0; b < B; ++b) {
        orc_table_sample_ld(gen, streams + b * 18, I, J, r, c, tab, J);
        if (orc_table_stat_ld(I, J, tab, J) <= threshold) ++count;
    }
    return count;
}
