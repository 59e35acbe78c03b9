/*
 * mrg_oracle.c -- plain, slow, obviously correct CPU oracle for the combined
 * multiple-recursive generators MRG32k3a and MRG31k3p run as many streams.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  Only tests/, the smoke check in __graft_entry__.py and the
 * cpu_baseline leg of bench.py may use it.  It shares no code, header, table
 * or constant generator with the GPU path.
 *
 * What it follows:
 *   - Section 2.1 (Creating streams) of Xu, Brown, L'Ecuyer, "clrng: A tool set
 *     for parallel random number generation on GPUs in R": the period is cut
 *     into disjoint pieces of length Z; a new stream's initial state is the
 *     creator state advanced by Z steps; the stream object keeps the current
 *     and the initial state; streams may be split into equally spaced
 *     substreams (RngStreams semantics, L'Ecuyer et al. 2002, which the paper
 *     cites for this).
 *   - Section 2.2 (Generating uniform random numbers): each step returns an
 *     integer z in [1, m1], scaled to (0,1) by 1/(m1+1); streams advance in
 *     place.
 *   - Section 3.1, Algorithm 1 (Box-Muller) and Section 3.2 (inverse
 *     transform for the exponential).
 *   - MRG32k3a itself is not defined in the paper (it is named in Sections 1,
 *     2 and 6 only).  Its definition is the published one: L'Ecuyer (1999),
 *     "Good parameters and implementations for combined multiple recursive
 *     random number generators", Operations Research 47(1), used by RngStreams.
 *   - MRG31k3p is the paper's own generator (Section 2, L'Ecuyer and Touzin
 *     2000).  It is here so that the generic machinery below can be checked
 *     against the values the paper prints for it.
 *
 * Arithmetic: recurrences in int64 with '%' (every term < 2^55), matrix
 * products in unsigned __int128 with '%', transforms in long double.  No
 * blocking, no fast reductions: a reader can check each line by eye.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Generator definitions                                                    */
/* ------------------------------------------------------------------------ */

enum { ORC_MRG32K3A = 1, ORC_MRG31K3P = 2 };
enum { ORC_UNIFORM = 0, ORC_NORMAL = 1, ORC_EXPONENTIAL = 2, ORC_RAW = 3 };
enum { ORC_F64 = 0, ORC_F32 = 1, ORC_U32 = 2 };

typedef struct {
    int64_t m[2];       /* moduli of the two components                      */
    int64_t a[2][3];    /* a[j][l-1] multiplies x_{j,n-l}, l = 1, 2, 3        */
    int newest_first;   /* order of the three words of a component in the
                           6-word external state: 0 = (x_{n-3}, x_{n-2},
                           x_{n-1}), 1 = (x_{n-1}, x_{n-2}, x_{n-3})         */
    int stream_log2;    /* streams are Z = 2^stream_log2 steps apart          */
    int substream_log2; /* substreams are 2^substream_log2 steps apart        */
} orc_gen;

/* MRG32k3a (L'Ecuyer 1999):
 *   x1,n = ( 1403580 x1,n-2 -  810728 x1,n-3) mod (2^32 - 209)
 *   x2,n = (  527612 x2,n-1 - 1370589 x2,n-3) mod (2^32 - 22853)
 * Streams 2^127 apart, substreams 2^76 apart (RngStreams).  The state is
 * kept oldest-first, the RngStreams convention.                            */
static const orc_gen GEN_MRG32K3A = {
    {4294967087LL, 4294944443LL},
    {{0, 1403580, -810728}, {527612, 0, -1370589}},
    0, 127, 76};

/* MRG31k3p (L'Ecuyer and Touzin 2000), the generator of the paper:
 *   x1,n = (2^22 x1,n-2 + (2^7 + 1) x1,n-3)  mod (2^31 - 1)
 *   x2,n = (2^15 x2,n-1 + (2^15 + 1) x2,n-3) mod (2^31 - 21069)
 * Streams Z = 2^134 apart (Section 2.1).  The words are printed newest-first
 * in the paper's stream table (Section 2.1).  Substreams 2^72 apart as in
 * clRNG.                                                                   */
static const orc_gen GEN_MRG31K3P = {
    {2147483647LL, 2147462579LL},
    {{0, 4194304, 129}, {32768, 0, 32769}},
    1, 134, 72};

static const orc_gen* gen_of(int id) {
    if (id == ORC_MRG32K3A) return &GEN_MRG32K3A;
    if (id == ORC_MRG31K3P) return &GEN_MRG31K3P;
    return NULL;
}

/* ------------------------------------------------------------------------ */
/* State order                                                              */
/* ------------------------------------------------------------------------ */

/* external 6-word state -> internal oldest-first (x_{n-3}, x_{n-2}, x_{n-1})
 * per component                                                            */
static void to_internal(const orc_gen* g, const uint32_t ext[6], int64_t x[2][3]) {
    for (int j = 0; j < 2; ++j)
        for (int i = 0; i < 3; ++i)
            x[j][i] = g->newest_first ? ext[3 * j + 2 - i] : ext[3 * j + i];
}

static void to_external(const orc_gen* g, int64_t x[2][3], uint32_t ext[6]) {
    for (int j = 0; j < 2; ++j)
        for (int i = 0; i < 3; ++i) {
            if (g->newest_first) ext[3 * j + 2 - i] = (uint32_t)x[j][i];
            else                 ext[3 * j + i]     = (uint32_t)x[j][i];
        }
}

/* ------------------------------------------------------------------------ */
/* One step of the recurrence and the output function                        */
/* ------------------------------------------------------------------------ */

/* x_{j,n} = (a1 x_{j,n-1} + a2 x_{j,n-2} + a3 x_{j,n-3}) mod m_j; the state
 * slides by one.  Returns the new value.                                   */
static int64_t comp_step(const orc_gen* g, int j, int64_t x[3]) {
    int64_t acc = g->a[j][0] * x[2] + g->a[j][1] * x[1] + g->a[j][2] * x[0];
    int64_t r = acc % g->m[j];
    if (r < 0) r += g->m[j];
    x[0] = x[1];
    x[1] = x[2];
    x[2] = r;
    return r;
}

/* z = x1 - x2 if x1 > x2, else x1 - x2 + m1: an integer in [1, m1]
 * (Section 2.2 states this range for the paper's generator).               */
uint64_t orc_output(int gen, uint64_t x1, uint64_t x2) {
    const orc_gen* g = gen_of(gen);
    if (x1 > x2) return x1 - x2;
    return (uint64_t)((int64_t)x1 - (int64_t)x2 + g->m[0]);
}

/* Advance the state one step (the step comes first, then the output: the
 * stream's initial state is never itself an output).                        */
static uint64_t step(const orc_gen* g, int64_t x[2][3]) {
    int64_t p1 = comp_step(g, 0, x[0]);
    int64_t p2 = comp_step(g, 1, x[1]);
    if (p1 > p2) return (uint64_t)(p1 - p2);
    return (uint64_t)(p1 - p2 + g->m[0]);
}

/* Advance an external state by one step and return z. */
uint64_t orc_step(int gen, uint32_t state[6]) {
    const orc_gen* g = gen_of(gen);
    int64_t x[2][3];
    to_internal(g, state, x);
    uint64_t z = step(g, x);
    to_external(g, x, state);
    return z;
}

/* ------------------------------------------------------------------------ */
/* Transforms                                                                */
/* ------------------------------------------------------------------------ */

/* u = z / (m1 + 1) in double precision (Section 2.2: the integer is scaled by
 * a constant 1/(m1+1)); NORM is 1/(m1+1) rounded to double, then one
 * multiply.                                                                 */
double orc_norm(int gen) {
    const orc_gen* g = gen_of(gen);
    return 1.0 / ((double)g->m[0] + 1.0);
}

double orc_uniform_f64(int gen, uint64_t z) { return (double)z * orc_norm(gen); }

/* The largest float not above u (round toward zero).  Round-to-nearest would
 * send m1/(m1+1) to 1.0 and leave (0,1).                                    */
float orc_f32_rz(double u) {
    float f = (float)u;
    if ((double)f > u) f = nextafterf(f, 0.0f);
    return f;
}

static const long double PI_L = 3.141592653589793238462643383279502884L;

/* Algorithm 1 (Box-Muller): R = sqrt(-2 log U1), Theta = 2 pi U2,
 * X = R cos Theta, Y = R sin Theta.  Evaluated in long double, rounded once
 * to double.                                                                */
void orc_box_muller(double u1, double u2, double* x, double* y) {
    long double r = sqrtl(-2.0L * logl((long double)u1));
    long double th = 2.0L * PI_L * (long double)u2;
    *x = (double)(r * cosl(th));
    *y = (double)(r * sinl(th));
}

/* Section 3.2: inverse transform of the exponential; E = -log(u) / rate
 * (the printed example of Section 3.2 uses u itself, not 1 - u).            */
double orc_exponential(double u, double rate) {
    return (double)(-logl((long double)u) / (long double)rate);
}

/* ------------------------------------------------------------------------ */
/* Matrix powers (jump-ahead), Section 2.1                                   */
/* ------------------------------------------------------------------------ */

/* One-step matrix on the oldest-first vector (x_{n-3}, x_{n-2}, x_{n-1}):
 * the next vector is (x_{n-2}, x_{n-1}, x_n).                               */
static void one_step_matrix(const orc_gen* g, int j, uint64_t A[9]) {
    int64_t m = g->m[j];
    memset(A, 0, 9 * sizeof(uint64_t));
    A[0 * 3 + 1] = 1;
    A[1 * 3 + 2] = 1;
    for (int l = 1; l <= 3; ++l) {
        int64_t c = g->a[j][l - 1] % m;
        if (c < 0) c += m;
        A[2 * 3 + (3 - l)] = (uint64_t)c;
    }
}

static void mat_mul(uint64_t m, const uint64_t A[9], const uint64_t B[9], uint64_t C[9]) {
    uint64_t T[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            unsigned __int128 acc = 0;
            for (int k = 0; k < 3; ++k)
                acc += (unsigned __int128)A[r * 3 + k] * B[k * 3 + c];
            T[r * 3 + c] = (uint64_t)(acc % m);
        }
    memcpy(C, T, sizeof(T));
}

/* A^e mod m for the one-step matrix of component `comp`; e is given as
 * `nwords` little-endian 64-bit words.  Plain square-and-multiply.          */
void orc_matpow(int gen, int comp, const uint64_t* e, int nwords, uint64_t out[9]) {
    const orc_gen* g = gen_of(gen);
    uint64_t m = (uint64_t)g->m[comp];
    uint64_t base[9], acc[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    one_step_matrix(g, comp, base);
    for (int w = 0; w < nwords; ++w)
        for (int b = 0; b < 64; ++b) {
            if ((e[w] >> b) & 1) mat_mul(m, acc, base, acc);
            mat_mul(m, base, base, base);
        }
    memcpy(out, acc, sizeof(acc));
}

/* v <- M v mod m on an oldest-first component vector. */
static void mat_vec(uint64_t m, const uint64_t M[9], int64_t v[3]) {
    int64_t t[3];
    for (int r = 0; r < 3; ++r) {
        unsigned __int128 acc = 0;
        for (int k = 0; k < 3; ++k) acc += (unsigned __int128)M[r * 3 + k] * (uint64_t)v[k];
        t[r] = (int64_t)(acc % m);
    }
    memcpy(v, t, sizeof(t));
}

/* Apply the two component matrices M[0], M[1] to an external state. */
static void apply(const orc_gen* g, uint64_t M[2][9], uint32_t state[6]) {
    int64_t x[2][3];
    to_internal(g, state, x);
    for (int j = 0; j < 2; ++j) mat_vec((uint64_t)g->m[j], M[j], x[j]);
    to_external(g, x, state);
}

/* Advance an external state by e steps (e as little-endian words). */
void orc_jump(int gen, uint32_t state[6], const uint64_t* e, int nwords) {
    const orc_gen* g = gen_of(gen);
    uint64_t M[2][9];
    for (int j = 0; j < 2; ++j) orc_matpow(gen, j, e, nwords, M[j]);
    apply(g, M, state);
}

/* Advance n external states, `stride` words apart, by the same e steps. */
void orc_jump_many(int gen, uint32_t* states, uint64_t n, uint64_t stride, const uint64_t* e,
                   int nwords) {
    const orc_gen* g = gen_of(gen);
    uint64_t M[2][9];
    for (int j = 0; j < 2; ++j) orc_matpow(gen, j, e, nwords, M[j]);
    for (uint64_t i = 0; i < n; ++i) apply(g, M, states + i * stride);
}

/* e = 2^k as little-endian words (k < 64 * 4). */
static void pow2_words(int k, uint64_t e[4]) {
    memset(e, 0, 4 * sizeof(uint64_t));
    e[k / 64] = (uint64_t)1 << (k % 64);
}

/* ------------------------------------------------------------------------ */
/* Seeds, creator and streams, Section 2.1                                   */
/* ------------------------------------------------------------------------ */

/* A seed is valid when its first three words are below m1, its last three
 * below m2, and neither triple is all zero (RngStreams' rule; the paper does
 * not state one).  Returns 1 when valid, 0 otherwise.                       */
int orc_seed_valid(int gen, const uint64_t seed[6]) {
    const orc_gen* g = gen_of(gen);
    for (int j = 0; j < 2; ++j) {
        int nonzero = 0;
        for (int i = 0; i < 3; ++i) {
            if (seed[3 * j + i] >= (uint64_t)g->m[j]) return 0;
            if (seed[3 * j + i] != 0) nonzero = 1;
        }
        if (!nonzero) return 0;
    }
    return 1;
}

/* Stream record: 18 words, (current, initial, substream start), 6 each. */
enum { ORC_CUR = 0, ORC_START = 6, ORC_SUB = 12, ORC_REC = 18 };

/* Create n streams one after another: each takes the creator state as its
 * initial (and current and substream) state, then the creator jumps ahead by
 * Z.  The creator is updated in place.                                      */
void orc_create_streams(int gen, uint32_t creator[6], uint64_t n, uint32_t* streams) {
    const orc_gen* g = gen_of(gen);
    uint64_t z[4], M[2][9];
    pow2_words(g->stream_log2, z);
    for (int j = 0; j < 2; ++j) orc_matpow(gen, j, z, 4, M[j]);  /* A^Z, once */
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t* s = streams + i * ORC_REC;
        memcpy(s + ORC_CUR, creator, 6 * sizeof(uint32_t));
        memcpy(s + ORC_START, creator, 6 * sizeof(uint32_t));
        memcpy(s + ORC_SUB, creator, 6 * sizeof(uint32_t));
        apply(g, M, creator);
    }
}

/* Substream operations (RngStreams semantics). */
void orc_next_substream(int gen, uint32_t* streams, uint64_t n) {
    const orc_gen* g = gen_of(gen);
    uint64_t e[4];
    pow2_words(g->substream_log2, e);
    orc_jump_many(gen, streams + ORC_SUB, n, ORC_REC, e, 4);
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t* s = streams + i * ORC_REC;
        memcpy(s + ORC_CUR, s + ORC_SUB, 6 * sizeof(uint32_t));
    }
    (void)g;
}

void orc_reset_substream(uint32_t* streams, uint64_t n) {
    for (uint64_t i = 0; i < n; ++i)
        memcpy(streams + i * ORC_REC + ORC_CUR, streams + i * ORC_REC + ORC_SUB, 6 * sizeof(uint32_t));
}

void orc_reset_stream(uint32_t* streams, uint64_t n) {
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t* s = streams + i * ORC_REC;
        memcpy(s + ORC_CUR, s + ORC_START, 6 * sizeof(uint32_t));
        memcpy(s + ORC_SUB, s + ORC_START, 6 * sizeof(uint32_t));
    }
}

void orc_advance(int gen, uint32_t* streams, uint64_t n, uint64_t k) {
    orc_jump_many(gen, streams + ORC_CUR, n, ORC_REC, &k, 1);
}

/* ------------------------------------------------------------------------ */
/* Generation                                                                */
/* ------------------------------------------------------------------------ */

static void put(void* out, uint64_t idx, int dtype, double v, uint64_t z, int dist) {
    if (dtype == ORC_U32) {
        ((uint32_t*)out)[idx] = (uint32_t)z;
    } else if (dtype == ORC_F64) {
        ((double*)out)[idx] = v;
    } else {
        /* float uniforms round toward zero; transformed values round to
           nearest from the double result                                  */
        ((float*)out)[idx] = dist == ORC_UNIFORM ? orc_f32_rz(v) : (float)v;
    }
}

/* cnt draws of one stream from state `cur` (advanced in place); draw k goes
 * to out[k * stride].  Uniform/raw: one step per draw.  Normal: draws 2p and
 * 2p+1 are X and Y of Algorithm 1 fed by the stream's steps 2p and 2p+1; an
 * odd count drops the last Y but still consumes its step.  Exponential: one
 * step per draw.                                                            */
int orc_stream_draws(int gen, uint32_t cur[6], uint64_t cnt, int dist, int dtype,
                     double param, void* out, uint64_t stride) {
    const orc_gen* g = gen_of(gen);
    if (!g) return -1;
    int64_t x[2][3];
    to_internal(g, cur, x);
    double norm = orc_norm(gen);
    if (dist == ORC_NORMAL) {
        for (uint64_t k = 0; k < cnt; k += 2) {
            double u1 = (double)step(g, x) * norm;
            double u2 = (double)step(g, x) * norm;
            double X, Y;
            orc_box_muller(u1, u2, &X, &Y);
            put(out, k * stride, dtype, X, 0, dist);
            if (k + 1 < cnt) put(out, (k + 1) * stride, dtype, Y, 0, dist);
        }
    } else {
        for (uint64_t k = 0; k < cnt; ++k) {
            uint64_t z = step(g, x);
            double u = (double)z * norm;
            double v = dist == ORC_EXPONENTIAL ? orc_exponential(u, param) : u;
            put(out, k * stride, dtype, v, z, dist);
        }
    }
    to_external(g, x, cur);
    return 0;
}

/* n numbers from S streams: stream s makes cnt_s = floor(n/S) + (s < n mod S)
 * draws, and draw k of stream s is out[k*S + s].  Streams [s_begin, s_end)
 * only, so that callers may split the work; the current states advance in
 * place.  `streams` points at stream 0's 18-word record.                    */
int orc_generate_range(int gen, uint32_t* streams, uint64_t S, uint64_t n, int dist,
                       int dtype, double param, void* out, uint64_t s_begin, uint64_t s_end) {
    if (S == 0) return n == 0 ? 0 : -1;
    uint64_t q = n / S, r = n % S;
    size_t esz = dtype == ORC_F64 ? 8 : 4;
    for (uint64_t s = s_begin; s < s_end && s < S; ++s) {
        uint64_t cnt = q + (s < r ? 1 : 0);
        int rc = orc_stream_draws(gen, streams + s * ORC_REC + ORC_CUR, cnt, dist, dtype, param,
                                  (char*)out + s * esz, S);
        if (rc) return rc;
    }
    return 0;
}

int orc_generate(int gen, uint32_t* streams, uint64_t S, uint64_t n, int dist, int dtype,
                 double param, void* out) {
    return orc_generate_range(gen, streams, S, n, dist, dtype, param, out, 0, S);
}

/* ------------------------------------------------------------------------ */
/* The paper's work-item geometry (Listing 1 of Section 2.2, Listing 2 of    */
/* Section 3.1)                                                              */
/* ------------------------------------------------------------------------ */

/* Stream of work-item (g0, g1) on a G0 x G1 lattice: uniforms and integers
 * take g0 + G0 g1 (Listing 1); normals take g0 G1 + g1 (Listing 2), and so do
 * exponentials (reading: the 2 x 4 matrix printed in Section 3.2 is only
 * reproduced with this index).                                             */
static uint64_t paper_stream(int dist, uint64_t g0, uint64_t g1, uint64_t G0, uint64_t G1) {
    if (dist == ORC_UNIFORM || dist == ORC_RAW) return g0 + G0 * g1;
    return g0 * G1 + g1;
}

/* An Nrow x Ncol output inside a row-major Nrow x Npad buffer.  Work-item
 * (g0, g1) owns the cells (r, c) with r = g0 (mod G0) and c = g1 (mod G1),
 * visits them rows ascending and, within a row, columns ascending, and puts
 * its next value at out[r * Npad + c].  For normals the work-items (g0, 2p)
 * and (g0, 2p + 1) form a pair: at each visit the first draws U1 from its
 * stream and the second draws U2 from its own; X goes to the first one's
 * cell, Y to the second one's (Algorithm 1; Listing 2 pairs the two through
 * local memory).  Normals need G1 and Ncol even, so that both members of a
 * pair make the same number of visits.  Streams not used stay as they are;
 * cells outside the Nrow x Ncol block are not written.  Returns -1 on an
 * invalid geometry (nothing is changed then).                               */
int orc_generate_paper(int gen, uint32_t* streams, uint64_t n_streams, uint64_t Nrow, uint64_t Ncol,
                       uint64_t Npad, uint64_t G0, uint64_t G1, int dist, int dtype, double param,
                       void* out) {
    const orc_gen* g = gen_of(gen);
    if (!g || G0 == 0 || G1 == 0 || Npad < Ncol || n_streams < G0 * G1) return -1;
    if (dist == ORC_NORMAL && (G1 % 2 || Ncol % 2)) return -1;
    const double norm = orc_norm(gen);
    for (uint64_t g0 = 0; g0 < G0; ++g0) {
        for (uint64_t g1 = 0; g1 < G1; ++g1) {
            if (dist == ORC_NORMAL && g1 % 2) continue; /* the pair's second member */
            uint32_t* a = streams + paper_stream(dist, g0, g1, G0, G1) * ORC_REC + ORC_CUR;
            int64_t xa[2][3], xb[2][3];
            to_internal(g, a, xa);
            uint32_t* b = NULL;
            if (dist == ORC_NORMAL) {
                b = streams + paper_stream(dist, g0, g1 + 1, G0, G1) * ORC_REC + ORC_CUR;
                to_internal(g, b, xb);
            }
            for (uint64_t r = g0; r < Nrow; r += G0) {
                for (uint64_t c = g1; c < Ncol; c += G1) {
                    if (dist == ORC_NORMAL) {
                        double u1 = (double)step(g, xa) * norm;
                        double u2 = (double)step(g, xb) * norm;
                        double X, Y;
                        orc_box_muller(u1, u2, &X, &Y);
                        put(out, r * Npad + c, dtype, X, 0, dist);
                        put(out, r * Npad + c + 1, dtype, Y, 0, dist);
                    } else {
                        uint64_t z = step(g, xa);
                        double u = (double)z * norm;
                        double v = dist == ORC_EXPONENTIAL ? orc_exponential(u, param) : u;
                        put(out, r * Npad + c, dtype, v, z, dist);
                    }
                }
            }
            to_external(g, xa, a);
            if (b) to_external(g, xb, b);
        }
    }
    return 0;
}
