// mrg_api.cpp -- the C ABI declared in include/mrg355.h.
//
// Every entry point validates all arguments before its first side effect, so
// a failing call launches nothing, writes nothing and leaves the creator
// unchanged.  Device work goes to the caller's hipStream_t.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "mrg355.h"
#include "mrg_internal.h"
#include "mrg_math.h"

using namespace mrg355;

static thread_local std::string g_err;

// Record the message of a failing call (thread-local) and return its status.
mrg_status mrg355_fail(mrg_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

namespace {

#define fail mrg355_fail

mrg_status ok() { return MRG_OK; }

mrg_status hip_fail(hipError_t e, const char* what) {
    return fail(MRG_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

mrg_status check_gen(mrg_generator gen) {
    if (gen == MRG_GEN_MRG32K3A || gen == MRG_GEN_MRG31K3P) return MRG_OK;
    return fail(MRG_E_INVALID_ARG, "unknown generator id %d", static_cast<int>(gen));
}

// The library's generator id (kGen32k3a / kGen31k3p) of a checked ABI id.
int gid(mrg_generator gen) { return gen == MRG_GEN_MRG32K3A ? kGen32k3a : kGen31k3p; }

// The seed / state validity rule: words 0-2 below m1, 3-5 below m2, neither
// triple all zero (the moduli of the generator).
bool state_valid(mrg_generator gen, const uint32_t s[6]) {
    const uint32_t m1 = gen == MRG_GEN_MRG32K3A ? kM1 : kP1;
    const uint32_t m2 = gen == MRG_GEN_MRG32K3A ? kM2 : kP2;
    if (s[0] >= m1 || s[1] >= m1 || s[2] >= m1) return false;
    if (s[3] >= m2 || s[4] >= m2 || s[5] >= m2) return false;
    if ((s[0] | s[1] | s[2]) == 0) return false;
    if ((s[3] | s[4] | s[5]) == 0) return false;
    return true;
}

constexpr char kMagic[4] = {'M', 'R', 'G', '3'};
constexpr uint32_t kFormatVersion = 1;
constexpr size_t kHeaderBytes = 4 + 4 + 4 + 4 + 8;
constexpr size_t kRecordBytes = sizeof(mrg_stream);

static_assert(sizeof(mrg_stream) == 72, "stream record is 18 words");

}  // namespace

extern "C" {

int mrg_abi_version(void) { return MRG_ABI_VERSION; }

const char* mrg_status_string(mrg_status st) {
    switch (st) {
        case MRG_OK: return "ok";
        case MRG_E_INVALID_ARG: return "invalid argument";
        case MRG_E_INVALID_SEED: return "invalid seed";
        case MRG_E_UNSUPPORTED: return "unsupported";
        case MRG_E_HIP: return "HIP runtime error";
        case MRG_E_NOMEM: return "out of memory / buffer too small";
        case MRG_E_CORRUPT_STATE: return "corrupt saved state";
        case MRG_E_BUSY: return "not done yet";
    }
    return "unknown status";
}

const char* mrg_last_error(void) { return g_err.c_str(); }

mrg_status mrg_seed_check(mrg_generator gen, const uint32_t seed[6]) {
    if (mrg_status st = check_gen(gen)) return st;
    if (!seed) return fail(MRG_E_INVALID_ARG, "seed is NULL");
    if (!state_valid(gen, seed))
        return fail(MRG_E_INVALID_SEED,
                    "seed words 0-2 must be < m1, words 3-5 < m2, and neither triple all zero");
    return ok();
}

mrg_status mrg_creator_init(mrg_generator gen, mrg_creator* creator, const uint32_t seed[6]) {
    if (!creator) return fail(MRG_E_INVALID_ARG, "creator is NULL");
    if (mrg_status st = mrg_seed_check(gen, seed)) return st;
    std::memcpy(creator->s, seed, sizeof(creator->s));
    return ok();
}

mrg_status mrg_streams_create_host(mrg_generator gen, mrg_creator* creator, size_t n,
                                   mrg_stream* host_out) {
    if (mrg_status st = check_gen(gen)) return st;
    if (!creator) return fail(MRG_E_INVALID_ARG, "creator is NULL");
    if (!state_valid(gen, creator->s)) return fail(MRG_E_INVALID_SEED, "creator holds an invalid state");
    if (n == 0) return ok();
    if (!host_out) return fail(MRG_E_INVALID_ARG, "host_out is NULL");
    // J = A^Z: one matrix-vector product per stream.
    uint32_t x[6];
    std::memcpy(x, creator->s, sizeof(x));
    for (size_t i = 0; i < n; ++i) {
        std::memcpy(host_out[i].cur, x, sizeof(x));
        std::memcpy(host_out[i].start, x, sizeof(x));
        std::memcpy(host_out[i].sub, x, sizeof(x));
        host_jump_pow2(gid(gen), x, 1, true);
    }
    std::memcpy(creator->s, x, sizeof(x));
    return ok();
}

mrg_status mrg_streams_create_device(mrg_generator gen, mrg_creator* creator, size_t n,
                                     mrg_stream* dev_out, hipStream_t stream) {
    if (mrg_status st = check_gen(gen)) return st;
    if (!creator) return fail(MRG_E_INVALID_ARG, "creator is NULL");
    if (!state_valid(gen, creator->s)) return fail(MRG_E_INVALID_SEED, "creator holds an invalid state");
    if (n == 0) return ok();
    if (!dev_out) return fail(MRG_E_INVALID_ARG, "dev_out is NULL");
    if (reinterpret_cast<uintptr_t>(dev_out) % 4) return fail(MRG_E_INVALID_ARG, "dev_out misaligned");
    if (n > (static_cast<size_t>(1) << 36)) return fail(MRG_E_INVALID_ARG, "n above 2^36");
    uint32_t next[6];
    std::memcpy(next, creator->s, sizeof(next));
    host_jump_pow2(gid(gen), next, static_cast<uint64_t>(n), true);
    hipError_t e = launch_create(gid(gen), reinterpret_cast<uint32_t*>(dev_out), n, creator->s, stream);
    if (e != hipSuccess) return hip_fail(e, "create_kernel launch");
    std::memcpy(creator->s, next, sizeof(next));
    return ok();
}

mrg_status mrg_streams_reset(mrg_generator gen, mrg_stream* dev, size_t n, mrg_reset_kind kind,
                             hipStream_t stream) {
    if (mrg_status st = check_gen(gen)) return st;
    if (kind != MRG_RESET_STREAM && kind != MRG_RESET_SUBSTREAM && kind != MRG_NEXT_SUBSTREAM)
        return fail(MRG_E_INVALID_ARG, "unknown reset kind %d", static_cast<int>(kind));
    if (n == 0) return ok();
    if (!dev) return fail(MRG_E_INVALID_ARG, "dev is NULL");
    if (reinterpret_cast<uintptr_t>(dev) % 4) return fail(MRG_E_INVALID_ARG, "dev misaligned");
    hipError_t e = launch_reset(gid(gen), reinterpret_cast<uint32_t*>(dev), n, static_cast<int>(kind), stream);
    if (e != hipSuccess) return hip_fail(e, "reset_kernel launch");
    return ok();
}

mrg_status mrg_streams_advance(mrg_generator gen, mrg_stream* dev, size_t n, uint64_t steps,
                               hipStream_t stream) {
    if (mrg_status st = check_gen(gen)) return st;
    if (n == 0 || steps == 0) return ok();
    if (!dev) return fail(MRG_E_INVALID_ARG, "dev is NULL");
    if (reinterpret_cast<uintptr_t>(dev) % 4) return fail(MRG_E_INVALID_ARG, "dev misaligned");
    hipError_t e = launch_advance(gid(gen), reinterpret_cast<uint32_t*>(dev), n, steps, stream);
    if (e != hipSuccess) return hip_fail(e, "advance_kernel launch");
    return ok();
}

// Validates a generate call's shape and launch cfg and fills L except its
// pointers.  *noop is set for n == 0 (nothing to launch).
static mrg_status generate_shape(mrg_generator gen, size_t n_streams, uint64_t n, mrg_dist dist,
                                 mrg_dtype dtype, double param, const mrg_launch_cfg* cfg, GenLaunch& L,
                                 bool* noop) {
    *noop = false;
    if (mrg_status st = check_gen(gen)) return st;
    if (dist != MRG_UNIFORM && dist != MRG_NORMAL && dist != MRG_EXPONENTIAL && dist != MRG_RAW)
        return fail(MRG_E_INVALID_ARG, "unknown distribution %d", static_cast<int>(dist));
    if (dtype != MRG_F64 && dtype != MRG_F32 && dtype != MRG_U32)
        return fail(MRG_E_INVALID_ARG, "unknown dtype %d", static_cast<int>(dtype));
    if ((dist == MRG_RAW) != (dtype == MRG_U32))
        return fail(MRG_E_INVALID_ARG, "MRG_RAW pairs with MRG_U32 only, and MRG_U32 with MRG_RAW only");
    if (dist == MRG_EXPONENTIAL && !(std::isfinite(param) && param > 0.0))
        return fail(MRG_E_INVALID_ARG, "exponential rate must be finite and > 0");
    L = GenLaunch{};
    if (cfg) {
        uint32_t b = cfg->block;
        if (b != 0 && b != 64 && b != 128 && b != 256 && b != 512 && b != 1024)
            return fail(MRG_E_INVALID_ARG, "block must be 64, 128, 256, 512 or 1024");
        if (cfg->arith > 2) return fail(MRG_E_INVALID_ARG, "arith must be 0, 1 or 2");
        if (cfg->nontemporal > 1) return fail(MRG_E_INVALID_ARG, "nontemporal must be 0 or 1");
        uint32_t spl = cfg->streams_per_lane;
        if (spl != 0 && spl != 1 && spl != 2 && spl != 4)
            return fail(MRG_E_INVALID_ARG, "streams_per_lane must be 0, 1, 2 or 4");
        if (cfg->xcd_remap > 1) return fail(MRG_E_INVALID_ARG, "xcd_remap must be 0 or 1");
        if (cfg->lockstep > 1) return fail(MRG_E_INVALID_ARG, "lockstep must be 0 or 1");
        L.block = static_cast<int>(b);
        L.chunk = cfg->chunk;
        L.nontemporal = static_cast<int>(cfg->nontemporal);
        L.arith = static_cast<int>(cfg->arith);
        L.spl = static_cast<int>(spl);
        L.xcd = static_cast<int>(cfg->xcd_remap);
        L.lock = static_cast<int>(cfg->lockstep);
    }
    if (n == 0) {
        *noop = true;
        return ok();
    }
    if (n_streams == 0) return fail(MRG_E_INVALID_ARG, "n_streams is 0 with n > 0");
    if (n_streams > (static_cast<size_t>(1) << 31)) return fail(MRG_E_INVALID_ARG, "n_streams above 2^31");
    if (n / n_streams >= (static_cast<uint64_t>(1) << 46))
        return fail(MRG_E_INVALID_ARG, "more than 2^46 draws per stream in one call");
    L.S = static_cast<uint32_t>(n_streams);
    L.q = n / n_streams;
    L.r = static_cast<uint32_t>(n % n_streams);
    L.dist = static_cast<int>(dist);
    L.dtype = static_cast<int>(dtype);
    L.param = dist == MRG_EXPONENTIAL ? 1.0 / param : 1.0;
    if (gen == MRG_GEN_MRG31K3P) L.arith = kArith31;  // its own engine; cfg->arith applies to MRG32k3a
    return ok();
}

mrg_status mrg_generate_ex(mrg_generator gen, mrg_stream* dev, size_t n_streams, uint64_t n,
                           mrg_dist dist, mrg_dtype dtype, double param, void* dev_out,
                           const mrg_launch_cfg* cfg, hipStream_t stream) {
    GenLaunch L;
    bool noop;
    if (mrg_status st = generate_shape(gen, n_streams, n, dist, dtype, param, cfg, L, &noop)) return st;
    if (noop) return ok();
    if (!dev || !dev_out) return fail(MRG_E_INVALID_ARG, "NULL stream or output pointer");
    const size_t esz = dtype == MRG_F64 ? 8 : 4;
    if (reinterpret_cast<uintptr_t>(dev_out) % esz)
        return fail(MRG_E_INVALID_ARG, "output not aligned to its element size");
    if (reinterpret_cast<uintptr_t>(dev) % 4) return fail(MRG_E_INVALID_ARG, "streams misaligned");
    L.streams = reinterpret_cast<uint32_t*>(dev);
    L.out = dev_out;
    plan_generate(L);
    hipError_t e = launch_generate(L, stream);
    if (e != hipSuccess) return hip_fail(e, "generate launch");
    return ok();
}

mrg_status mrg_generate_plan(mrg_generator gen, size_t n_streams, uint64_t n, mrg_dist dist, mrg_dtype dtype,
                             double param, const mrg_launch_cfg* cfg, mrg_launch_cfg* resolved) {
    if (!resolved) return fail(MRG_E_INVALID_ARG, "NULL resolved cfg");
    GenLaunch L;
    bool noop;
    if (mrg_status st = generate_shape(gen, n_streams, n, dist, dtype, param, cfg, L, &noop)) return st;
    *resolved = mrg_launch_cfg{};
    if (noop) return ok();
    // an output address aligned to 256 bytes, as device allocations are; only
    // its alignment is looked at
    L.out = reinterpret_cast<void*>(static_cast<uintptr_t>(256));
    plan_generate(L);
    resolved->block = static_cast<uint32_t>(L.block);
    resolved->chunk = L.chunk;
    resolved->nontemporal = static_cast<uint32_t>(L.nontemporal);
    resolved->arith = L.arith == kArith31 ? 0u : static_cast<uint32_t>(L.arith);
    resolved->streams_per_lane = static_cast<uint32_t>(L.spl);
    resolved->xcd_remap = static_cast<uint32_t>(L.xcd);
    resolved->lockstep = static_cast<uint32_t>(L.lock);
    return ok();
}

mrg_status mrg_generate(mrg_generator gen, mrg_stream* dev, size_t n_streams, uint64_t n,
                        mrg_dist dist, mrg_dtype dtype, double param, void* dev_out,
                        hipStream_t stream) {
    return mrg_generate_ex(gen, dev, n_streams, n, dist, dtype, param, dev_out, nullptr, stream);
}

mrg_status mrg_generate_paper(mrg_generator gen, mrg_stream* dev, size_t n_streams, uint64_t nrow, uint64_t ncol,
                              uint64_t npad, uint32_t g0size, uint32_t g1size, mrg_dist dist, mrg_dtype dtype,
                              double param, void* dev_out, hipStream_t stream) {
    if (mrg_status st = check_gen(gen)) return st;
    if (dist != MRG_UNIFORM && dist != MRG_NORMAL && dist != MRG_EXPONENTIAL && dist != MRG_RAW)
        return fail(MRG_E_INVALID_ARG, "unknown distribution %d", static_cast<int>(dist));
    if (dtype != MRG_F64 && dtype != MRG_F32 && dtype != MRG_U32)
        return fail(MRG_E_INVALID_ARG, "unknown dtype %d", static_cast<int>(dtype));
    if ((dist == MRG_RAW) != (dtype == MRG_U32))
        return fail(MRG_E_INVALID_ARG, "MRG_RAW pairs with MRG_U32 only, and MRG_U32 with MRG_RAW only");
    if (dist == MRG_EXPONENTIAL && !(std::isfinite(param) && param > 0.0))
        return fail(MRG_E_INVALID_ARG, "exponential rate must be finite and > 0");
    if (g0size == 0 || g1size == 0) return fail(MRG_E_INVALID_ARG, "the work-item lattice must be non-empty");
    if (n_streams > (static_cast<size_t>(1) << 31)) return fail(MRG_E_INVALID_ARG, "n_streams above 2^31");
    if (static_cast<uint64_t>(g0size) * g1size > n_streams)
        return fail(MRG_E_INVALID_ARG, "%u x %u work-items need as many streams, %zu given", g0size, g1size,
                    n_streams);
    if (npad < ncol) return fail(MRG_E_INVALID_ARG, "npad below ncol");
    if (nrow >= (1ull << 31) || ncol >= (1ull << 31)) return fail(MRG_E_INVALID_ARG, "nrow and ncol below 2^31");
    if (nrow && npad > (1ull << 62) / nrow) return fail(MRG_E_INVALID_ARG, "nrow * npad too large");
    if (dist == MRG_NORMAL && (g1size % 2 || ncol % 2))
        return fail(MRG_E_INVALID_ARG, "normals pair work-items along the second dimension: G1 and ncol must be even");
    if (nrow == 0 || ncol == 0) return ok();
    if (!dev || !dev_out) return fail(MRG_E_INVALID_ARG, "NULL stream or output pointer");
    const size_t esz = dtype == MRG_F64 ? 8 : 4;
    if (reinterpret_cast<uintptr_t>(dev_out) % esz)
        return fail(MRG_E_INVALID_ARG, "output not aligned to its element size");
    if (reinterpret_cast<uintptr_t>(dev) % 4) return fail(MRG_E_INVALID_ARG, "streams misaligned");
    PaperLaunch L{};
    L.streams = reinterpret_cast<uint32_t*>(dev);
    L.out = dev_out;
    L.npad = npad;
    L.nrow = static_cast<uint32_t>(nrow);
    L.ncol = static_cast<uint32_t>(ncol);
    L.G0 = g0size;
    L.G1 = g1size;
    L.dist = static_cast<int>(dist);
    L.dtype = static_cast<int>(dtype);
    L.param = dist == MRG_EXPONENTIAL ? 1.0 / param : 1.0;
    plan_paper(L, gid(gen));
    hipError_t e = launch_paper(L, gid(gen), stream);
    if (e != hipSuccess) return hip_fail(e, "paper-geometry launch");
    return ok();
}

mrg_status mrg_tables_sample(mrg_generator gen, mrg_stream* dev_streams, size_t n, const int32_t* dev_I,
                             const int32_t* dev_J, const int32_t* dev_rows, const int32_t* dev_cols,
                             int32_t* dev_tables, double* dev_stats, hipStream_t stream) {
    if (mrg_status st = check_gen(gen)) return st;
    if (n == 0) return ok();
    if (!dev_streams || !dev_I || !dev_J || !dev_rows || !dev_cols || !dev_tables)
        return fail(MRG_E_INVALID_ARG, "NULL pointer");
    if (n > (static_cast<size_t>(1) << 31)) return fail(MRG_E_INVALID_ARG, "n above 2^31");
    if (reinterpret_cast<uintptr_t>(dev_streams) % 4 || reinterpret_cast<uintptr_t>(dev_tables) % 4 ||
        reinterpret_cast<uintptr_t>(dev_I) % 4 || reinterpret_cast<uintptr_t>(dev_J) % 4 ||
        reinterpret_cast<uintptr_t>(dev_rows) % 4 || reinterpret_cast<uintptr_t>(dev_cols) % 4 ||
        reinterpret_cast<uintptr_t>(dev_stats) % 8)
        return fail(MRG_E_INVALID_ARG, "misaligned pointer");
    hipError_t e = launch_tables(gid(gen), reinterpret_cast<uint32_t*>(dev_streams), n, dev_I, dev_J, dev_rows, dev_cols,
                                 dev_tables, dev_stats, stream);
    if (e != hipSuccess) return hip_fail(e, "tables launch");
    return ok();
}

mrg_status mrg_fisher_sim(mrg_generator gen, mrg_stream* dev_streams, uint64_t B, int I, int J,
                          const int32_t* observed, uint64_t* dev_count, double* dev_stats,
                          double* observed_stat, hipStream_t stream) {
    if (mrg_status st = check_gen(gen)) return st;
    if (!observed || !dev_count) return fail(MRG_E_INVALID_ARG, "NULL observed table or count");
    if (I < 1 || J < 1 || I > kFisherMaxDim || J > kFisherMaxDim)
        return fail(MRG_E_INVALID_ARG, "table shape must be 1..%d x 1..%d", kFisherMaxDim, kFisherMaxDim);
    if (B && !dev_streams) return fail(MRG_E_INVALID_ARG, "NULL streams");
    if (B > (static_cast<uint64_t>(1) << 31)) return fail(MRG_E_INVALID_ARG, "B above 2^31");
    if (reinterpret_cast<uintptr_t>(dev_count) % 8 || reinterpret_cast<uintptr_t>(dev_stats) % 8 ||
        reinterpret_cast<uintptr_t>(dev_streams) % 4)
        return fail(MRG_E_INVALID_ARG, "misaligned pointer");
    // margins summed in 64 bits and narrowed only after the total is known
    // to be at most 2^20 (entries up to 2^31 - 1 cannot overflow them)
    int64_t r64[kFisherMaxDim] = {0}, c64[kFisherMaxDim] = {0};
    int64_t total = 0;
    for (int i = 0; i < I; ++i)
        for (int j = 0; j < J; ++j) {
            const int32_t v = observed[i * J + j];
            if (v < 0) return fail(MRG_E_INVALID_ARG, "negative entry in the observed table");
            r64[i] += v;
            c64[j] += v;
            total += v;
        }
    if (total > kTableMaxTotal) return fail(MRG_E_INVALID_ARG, "grand total above 2^20");
    int32_t r[kFisherMaxDim] = {0}, c[kFisherMaxDim] = {0};
    for (int i = 0; i < I; ++i) r[i] = static_cast<int32_t>(r64[i]);
    for (int j = 0; j < J; ++j) c[j] = static_cast<int32_t>(c64[j]);
    double stat = 0.0;  // -sum log(n!), row-major, from the same values as the device table
    for (int i = 0; i < I; ++i)
        for (int j = 0; j < J; ++j) stat -= host_log_factorial(observed[i * J + j]);
    const double threshold = stat / (1.0 + 64.0 * DBL_EPSILON);
    hipError_t e = launch_fisher(gid(gen), reinterpret_cast<uint32_t*>(dev_streams), B, I, J, r, c, threshold,
                                 reinterpret_cast<unsigned long long*>(dev_count), dev_stats, stream);
    if (e != hipSuccess) return hip_fail(e, "fisher launch");
    if (observed_stat) *observed_stat = stat;
    return ok();
}

double mrg_fisher_pvalue(uint64_t count, uint64_t B) {
    return (1.0 + static_cast<double>(count)) / (static_cast<double>(B) + 1.0);
}

mrg_status mrg_transform_accuracy(mrg_generator gen, mrg_check_fn fn, uint64_t z_begin, uint64_t z_end,
                                  uint64_t* dev_result, hipStream_t stream) {
    if (mrg_status st = check_gen(gen)) return st;
    if (static_cast<int>(fn) < MRG_CHECK_LOG || static_cast<int>(fn) > MRG_CHECK_COSPI_F32OUT)
        return fail(MRG_E_INVALID_ARG, "unknown function %d", static_cast<int>(fn));
    const uint64_t m1 = gen == MRG_GEN_MRG32K3A ? kM1 : kP1;
    if (z_begin < 1 || z_begin > z_end || z_end > m1 + 1)
        return fail(MRG_E_INVALID_ARG, "z range must satisfy 1 <= z_begin <= z_end <= m1 + 1");
    if (!dev_result || reinterpret_cast<uintptr_t>(dev_result) % 8)
        return fail(MRG_E_INVALID_ARG, "dev_result is NULL or misaligned");
    hipError_t e = launch_accuracy(gid(gen), static_cast<int>(fn), z_begin, z_end,
                                   reinterpret_cast<unsigned long long*>(dev_result), stream);
    if (e != hipSuccess) return hip_fail(e, "accuracy launch");
    return ok();
}

mrg_status mrg_store_ceiling(size_t n_streams, uint64_t n, mrg_dtype dtype, void* dev_out, hipStream_t stream) {
    if (dtype != MRG_F64 && dtype != MRG_F32) return fail(MRG_E_INVALID_ARG, "dtype must be MRG_F64 or MRG_F32");
    GenLaunch L;
    bool noop;
    if (mrg_status st = generate_shape(MRG_GEN_MRG32K3A, n_streams, n, MRG_UNIFORM, dtype, 1.0, nullptr, L, &noop))
        return st;
    if (noop) return ok();
    if (n % n_streams) return fail(MRG_E_INVALID_ARG, "n must be a multiple of n_streams");
    if (!dev_out) return fail(MRG_E_INVALID_ARG, "dev_out is NULL");
    const size_t esz = dtype == MRG_F64 ? 8 : 4;
    if (reinterpret_cast<uintptr_t>(dev_out) % esz)
        return fail(MRG_E_INVALID_ARG, "output not aligned to its element size");
    L.out = dev_out;
    plan_generate(L);
    hipError_t e = launch_store_ceiling(L, stream);
    if (e != hipSuccess) return hip_fail(e, "store ceiling launch");
    return ok();
}

mrg_status mrg_streams_export_size(size_t n, int with_creator, size_t* bytes) {
    if (!bytes) return fail(MRG_E_INVALID_ARG, "bytes is NULL");
    if (n > (SIZE_MAX - kHeaderBytes - 24) / kRecordBytes) return fail(MRG_E_INVALID_ARG, "n too large");
    *bytes = kHeaderBytes + n * kRecordBytes + (with_creator ? 24 : 0);
    return ok();
}

mrg_status mrg_streams_export(mrg_generator gen, const mrg_stream* dev, size_t n,
                              const mrg_creator* creator, void* host_buf, size_t cap, size_t* len,
                              hipStream_t stream) {
    if (mrg_status st = check_gen(gen)) return st;
    if (!host_buf || !len) return fail(MRG_E_INVALID_ARG, "NULL host buffer or length pointer");
    if (n && !dev) return fail(MRG_E_INVALID_ARG, "dev is NULL");
    size_t need = 0;
    if (mrg_status st = mrg_streams_export_size(n, creator != nullptr, &need)) return st;
    if (cap < need) return fail(MRG_E_NOMEM, "export needs %zu bytes, capacity is %zu", need, cap);
    unsigned char* p = static_cast<unsigned char*>(host_buf);
    const uint32_t version = kFormatVersion, g = static_cast<uint32_t>(gen);
    const uint32_t flags = creator ? 1u : 0u;
    const uint64_t n64 = n;
    if (n) {
        hipError_t e = hipMemcpyAsync(p + kHeaderBytes, dev, n * kRecordBytes, hipMemcpyDeviceToHost, stream);
        if (e != hipSuccess) return hip_fail(e, "export copy");
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "export synchronize");
    }
    std::memcpy(p, kMagic, 4);
    std::memcpy(p + 4, &version, 4);
    std::memcpy(p + 8, &g, 4);
    std::memcpy(p + 12, &flags, 4);
    std::memcpy(p + 16, &n64, 8);
    if (creator) std::memcpy(p + kHeaderBytes + n * kRecordBytes, creator->s, 24);
    *len = need;
    return ok();
}

mrg_status mrg_streams_import(mrg_generator gen, const void* host_buf, size_t len, mrg_stream* dev,
                              size_t n, size_t* n_out, mrg_creator* creator, hipStream_t stream) {
    if (mrg_status st = check_gen(gen)) return st;
    if (!host_buf) return fail(MRG_E_INVALID_ARG, "host_buf is NULL");
    const unsigned char* p = static_cast<const unsigned char*>(host_buf);
    if (len < kHeaderBytes) return fail(MRG_E_CORRUPT_STATE, "buffer shorter than the header");
    if (std::memcmp(p, kMagic, 4) != 0) return fail(MRG_E_CORRUPT_STATE, "bad magic");
    uint32_t version, g, flags;
    uint64_t cnt;
    std::memcpy(&version, p + 4, 4);
    std::memcpy(&g, p + 8, 4);
    std::memcpy(&flags, p + 12, 4);
    std::memcpy(&cnt, p + 16, 8);
    if (version != kFormatVersion) return fail(MRG_E_CORRUPT_STATE, "unsupported format version %u", version);
    if (g != static_cast<uint32_t>(gen)) return fail(MRG_E_CORRUPT_STATE, "saved generator id %u differs", g);
    if (flags > 1) return fail(MRG_E_CORRUPT_STATE, "unknown flags 0x%x", flags);
    if (cnt > (SIZE_MAX - kHeaderBytes - 24) / kRecordBytes) return fail(MRG_E_CORRUPT_STATE, "bad count");
    const size_t need = kHeaderBytes + cnt * kRecordBytes + (flags ? 24 : 0);
    if (len != need) return fail(MRG_E_CORRUPT_STATE, "length %zu does not match %zu", len, need);
    uint32_t tmp[6];
    for (uint64_t i = 0; i < cnt * 3; ++i) {  // cur, start and sub of every record
        std::memcpy(tmp, p + kHeaderBytes + i * 24, 24);
        if (!state_valid(gen, tmp))
            return fail(MRG_E_CORRUPT_STATE, "record %llu holds an invalid state",
                        static_cast<unsigned long long>(i / 3));
    }
    uint32_t cre[6] = {0, 0, 0, 0, 0, 0};
    if (flags) {
        std::memcpy(cre, p + kHeaderBytes + cnt * kRecordBytes, 24);
        if (!state_valid(gen, cre)) return fail(MRG_E_CORRUPT_STATE, "saved creator is invalid");
    }
    if (cnt > n) return fail(MRG_E_NOMEM, "buffer holds %llu streams, room for %zu",
                             static_cast<unsigned long long>(cnt), n);
    if (cnt && !dev) return fail(MRG_E_INVALID_ARG, "dev is NULL");
    if (cnt) {
        hipError_t e = hipMemcpyAsync(dev, p + kHeaderBytes, cnt * kRecordBytes, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return hip_fail(e, "import copy");
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "import synchronize");
    }
    if (n_out) *n_out = cnt;
    if (creator && flags) std::memcpy(creator->s, cre, 24);
    return ok();
}

}  // extern "C"
