// mrg_internal.h -- interface between the C-ABI layer (mrg_api.cpp) and the
// gfx950 kernels (mrg_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <vector>

namespace mrg355 {

enum Dist { kUniform = 0, kNormal = 1, kExponential = 2, kRaw = 3 };
enum DType { kF64 = 0, kF32 = 1, kU32 = 2 };
// kArith31 is the MRG31k3p engine (set by the library for that generator).
enum Arith { kArithAuto = 0, kArithInt = 1, kArithF64 = 2, kArith31 = 3 };

// One plain generation launch over S streams (see mrg_generate).
struct GenLaunch {
    uint32_t* streams;   // S records of 18 words; `cur` is read and written
    void* out;           // dense n elements
    uint64_t q;          // floor(n / S)
    uint32_t S;          // streams
    uint32_t r;          // n mod S
    uint32_t chunk;      // units (draws; normal: pairs) per work-item
    uint32_t n_chunks;   // work-items per stream
    double param;        // 1/rate for exponentials
    int dist, dtype, arith, block, nontemporal;
    int spl;             // streams per lane (1, 2, 4); 0 = automatic
    int xcd;             // 1 = XCD-contiguous block order
    uint64_t offset;     // steps every stream is advanced before its first draw
    int no_writeback;    // 1 = leave the stream records untouched (served requests)
    int lock;            // 1 = the waves of a block write each row together (barrier per row)
};

// Resolve chunk/n_chunks/block/arith left at 0 to the automatic choice.
void plan_generate(GenLaunch& L);

// ---------------------------------------------------------------- batching
// Kinds of tile the persistent kernel can run (dist, dtype, streams per lane).
enum BatchKind {
    kBUniF64x1, kBUniF64x2, kBUniF32x1, kBUniF32x4, kBRawU32x1, kBRawU32x4,
    kBNormF64, kBNormF32, kBExpF64, kBExpF32,
    kBNormF64x2, kBNormF32x2, kBExpF64x2, kBExpF32x2, kBKinds
};

struct BatchReq {       // one request, static for a plan
    GenLaunch L;        // its launch description (chunk = tile units)
    uint32_t n_tiles;
    uint32_t kind;
};

struct BatchTile {      // a wave's unit of work
    uint32_t req, sblk, chunk, pad;
};
constexpr uint32_t kNoRequest = 0xffffffffu;  // BatchTile.req of the padding of a short gang

struct BatchSlot {      // per-request counters, reset by every launch
    uint32_t remaining; // tiles not finished
    uint32_t done;      // 1 once every tile has stored its output
    uint64_t t_done;    // device real-time clock (100 MHz) at completion
};

// Tile classes: each has its own queue and its own worker loop.
enum BatchClass { kClsNormal = 0, kClsExp = 1, kClsPlain = 2, kClasses = 3 };

inline int batch_kind_class(int kind) {
    if (kind == kBNormF64 || kind == kBNormF32 || kind == kBNormF64x2 || kind == kBNormF32x2) return kClsNormal;
    if (kind == kBExpF64 || kind == kBExpF32 || kind == kBExpF64x2 || kind == kBExpF32x2) return kClsExp;
    return kClsPlain;
}

constexpr int kXcdQueues = 8;  // gang mode: one gang queue per XCD (block b runs on XCD b mod 8)

struct BatchHeader {    // at workspace offset 0, reset by every launch
    uint32_t queue[kXcdQueues];  // next tile (class queues) or gang (per XCD) to hand out
    uint64_t t_start;   // device real-time clock when the persistent kernel started
};

struct BatchLaunch {    // kernel arguments
    BatchHeader* head;
    BatchSlot* slots;
    BatchSlot* host_slots;    // optional copy of done/t_done in host-mapped memory
    const BatchReq* reqs;
    const BatchTile* tiles;
    const uint32_t* fin_req;  // requests split over chunks (state advanced afterwards)
    const uint64_t* fin_pre;  // prefix sums of their stream counts
    uint32_t n_req, n_tiles, n_fin;
    uint32_t tile_lo[kClasses + 1];   // class c owns tiles [tile_lo[c], tile_lo[c+1])
    uint32_t block_lo[kClasses + 1];  // and blocks [block_lo[c], block_lo[c+1])
    uint32_t wpb;                     // waves per block of the persistent kernel
    uint64_t fin_total;
    uint32_t n_gangs;                 // gang mode: tiles[g*wpb .. g*wpb+wpb-1] is gang g; 0 = class queues
    uint32_t grid;                    // blocks of the persistent kernel
    uint32_t narrow;                  // gang mode: 1 = every tile is of one stream per lane
    uint32_t xq_lo[kXcdQueues + 1];   // gang mode: XCD x's queue holds gangs [xq_lo[x], xq_lo[x+1])
};

hipError_t launch_batch(const BatchLaunch& B, unsigned grid, unsigned block, hipStream_t s);
int batch_gang_blocks_per_cu(unsigned block, bool narrow);
inline bool batch_kind_narrow(int kind) {
    return kind == kBUniF64x1 || kind == kBUniF32x1 || kind == kBRawU32x1 || kind == kBNormF64 || kind == kBNormF32 ||
           kind == kBExpF64 || kind == kBExpF32;
}

}  // namespace mrg355

#include "mrg355.h"

namespace mrg355 {

// A request of a plan: the public request plus where its streams start.
struct PlanReq {
    mrg_request q;
    uint64_t offset;    // steps each stream advances before its first draw
    int no_writeback;   // 1 = do not write the stream records back
    uint32_t split;     // > 0: cut each stream block into about this many tiles
                        // (at least 96 units each), for latency; 0 = tile_units
};

mrg_status plan_internal(const std::vector<PlanReq>& reqs, uint32_t tile_units, mrg_batch_plan** out);
size_t plan_bytes(const mrg_batch_plan* P);
size_t plan_table_offset(const mrg_batch_plan* P);
void plan_pack_tables(const mrg_batch_plan* P, char* host);
mrg_status plan_launch(const mrg_batch_plan* P, void* ws, BatchSlot* host_slots, hipStream_t stream);
int batch_kind(int dist, int dtype, int spl);
int device_cu_count();
int batch_blocks_per_cu();
hipError_t launch_generate(const GenLaunch& L, hipStream_t s);

// gen: kGen32k3a or kGen31k3p (mrg_math.h).
hipError_t launch_create(int gen, uint32_t* out, uint64_t n, const uint32_t creator[6], hipStream_t s);
hipError_t launch_reset(int gen, uint32_t* streams, uint64_t n, int kind, hipStream_t s);
hipError_t launch_advance(int gen, uint32_t* streams, uint64_t n, uint64_t steps, hipStream_t s);

// Contingency tables (Section 4).
constexpr int kFisherMaxDim = 32;
constexpr int64_t kTableMaxTotal = 1 << 20;  // grand total of one table at most
hipError_t launch_tables(int gen, uint32_t* streams, uint64_t n, const int32_t* I, const int32_t* J, const int32_t* rows,
                         const int32_t* cols, int32_t* tabs, double* stats, hipStream_t s);
double host_log_factorial(int64_t k);  // lgamma(k+1) in long double, rounded to double
hipError_t launch_fisher(int gen, uint32_t* streams, uint64_t B, int I, int J, const int32_t* r, const int32_t* c,
                         double threshold, unsigned long long* count, double* stats, hipStream_t s);

// The paper's work-item geometry (Listing 1 / Listing 2): see mrg_generate_paper.
struct PaperLaunch {
    uint32_t* streams;
    void* out;
    uint64_t npad;       // row stride of out, in elements
    uint32_t nrow, ncol; // the block written
    uint32_t G0, G1;     // work-item lattice
    uint32_t lanes_g1;   // G1, or G1/2 pairs for normals
    uint32_t rows_per;   // a lane's chunk: rows_per of its work-item's rows ...
    uint32_t n_rb;       // ... in n_rb row blocks,
    uint32_t cols_per;   // and cols_per of each row's visits (cols_per < all only with rows_per = 1) ...
    uint32_t n_cb;       // ... in n_cb column blocks
    int dist, dtype;
    double param;        // 1/rate for exponentials
};
void plan_paper(PaperLaunch& L, int gen);
hipError_t launch_paper(const PaperLaunch& L, int gen, hipStream_t s);

// Diagnostics (mrg_selfcheck.hip, mrg_kernels.hip).
constexpr int kAccuracyBins = 5;   // distances 0, 1, 2, 3 and >= 4 ulp
constexpr int kAccuracyWords = 8;  // bins, the packed worst case, two reserved words
hipError_t launch_accuracy(int gen, int fn, uint64_t z0, uint64_t z1, unsigned long long* res, hipStream_t s);
hipError_t launch_store_ceiling(const GenLaunch& L, hipStream_t s);

// Host-side jump math (same tables the device uses).
void host_jump_pow2(int gen, uint32_t state[6], uint64_t k, bool stream_tables);  // A^(k [* Z]) state

}  // namespace mrg355
