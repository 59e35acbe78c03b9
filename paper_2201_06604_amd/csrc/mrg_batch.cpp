// mrg_batch.cpp -- host side of batched generation: plans (tiles, workspace
// layout), upload, launch, completion times and the autotuner.
//
// A request is the argument list of one mrg_generate call.  A plan cuts every
// request into tiles -- (request, block of 64*SPL streams, chunk of at most
// tile_units draw units) -- and orders them by estimated cost, longest first,
// so that the persistent kernel's waves, which take tiles from one atomic
// counter, finish together.  Each tile runs exactly the code of the plain
// generate kernel for its piece, so results are identical to per-request
// launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "mrg355.h"
#include "mrg_internal.h"
#include "mrg_math.h"

using namespace mrg355;

mrg_status mrg355_fail(mrg_status st, const char* fmt, ...);  // mrg_api.cpp

struct mrg_batch_plan {
    mrg_generator gen;
    std::vector<mrg355::PlanReq> user;
    uint32_t tile_units;
    uint32_t waves_per_simd;
    uint32_t wide;
    uint32_t gang;  // 1 = class queues of wave tiles; 2, 4, 8 = gangs of that many waves
    std::vector<BatchReq> reqs;
    std::vector<BatchTile> tiles;
    uint32_t tile_lo[kClasses + 1];
    double cls_cost[kClasses];
    uint32_t n_gangs;  // gang mode: tiles holds n_gangs * gang entries (padding: req = kNoRequest)
    uint32_t narrow;   // every request runs one stream per lane (the narrow gang kernel serves it)
    uint32_t xq_lo[kXcdQueues + 1];  // gang mode: the gangs of each XCD's queue
    std::vector<uint32_t> fin_req;
    std::vector<uint64_t> fin_pre;
    uint64_t fin_total;
    size_t off_slots, off_reqs, off_tiles, off_fin_req, off_fin_pre, bytes;
    std::vector<char> packed;  // the static tables as uploaded (workspace bytes from off_reqs on)
};

namespace {

// The shape the autotuner picks for the 4,096-request mix of lengths 10^3 to
// 10^7 and 64 to 1,024 streams: gangs of 8 waves, one stream per lane (the
// narrow kernel), 256-unit tiles, 4 waves per SIMD.
constexpr uint32_t kDefaultTileUnits = 256;
constexpr uint32_t kDefaultWavesPerSimd = 4;
constexpr uint32_t kDefaultGang = 8;
constexpr unsigned kBatchBlock = 256;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t esz_of(mrg_dtype dt) { return dt == MRG_F64 ? 8 : 4; }

// Estimated time of one draw unit of one stream, relative units, from the
// rates of plain launches over many streams: about 700 G f64 uniforms/s
// (store-bound), 1.4 T f32 uniforms/s, 325 G normals/s and 300 G
// exponentials/s (the transcendental rates before the library's own log and
// sin/cos).  They set the order of the tiles and each class's share of the
// blocks.  Weighting the VALU-bound classes this heavily is deliberate: an
// A/B on the 4,096-request mix against the rates each class reaches inside
// the batch (uniforms ~330-440 G/s, normals ~280-330, exponentials
// ~335-450) gave 10.53-10.55 ms against 10.77-10.80 ms, since store-bound
// uniform tiles run well beside the transform-heavy ones.
double unit_cost(int dist, int dtype) {
    switch (dist) {
        case kNormal: return 2.0 / 325.0;  // per pair
        case kExponential: return 1.0 / 300.0;
        default: return dtype == kF64 ? 1.0 / 700.0 : 1.0 / 1400.0;
    }
}

mrg_status validate_request(const mrg_request& q, size_t i) {
    const mrg_dist dist = q.dist;
    const mrg_dtype dtype = q.dtype;
    if (dist != MRG_UNIFORM && dist != MRG_NORMAL && dist != MRG_EXPONENTIAL && dist != MRG_RAW)
        return mrg355_fail(MRG_E_INVALID_ARG, "request %zu: unknown distribution", i);
    if (dtype != MRG_F64 && dtype != MRG_F32 && dtype != MRG_U32)
        return mrg355_fail(MRG_E_INVALID_ARG, "request %zu: unknown dtype", i);
    if ((dist == MRG_RAW) != (dtype == MRG_U32))
        return mrg355_fail(MRG_E_INVALID_ARG, "request %zu: MRG_RAW pairs with MRG_U32 only", i);
    if (dist == MRG_EXPONENTIAL && !(std::isfinite(q.param) && q.param > 0.0))
        return mrg355_fail(MRG_E_INVALID_ARG, "request %zu: exponential rate must be finite and > 0", i);
    if (q.n == 0) return MRG_OK;
    if (q.n_streams == 0) return mrg355_fail(MRG_E_INVALID_ARG, "request %zu: no streams", i);
    if (q.n_streams > (1u << 31)) return mrg355_fail(MRG_E_INVALID_ARG, "request %zu: too many streams", i);
    if (q.n / q.n_streams >= (static_cast<uint64_t>(1) << 46))
        return mrg355_fail(MRG_E_INVALID_ARG, "request %zu: more than 2^46 draws per stream", i);
    if (!q.streams || !q.out) return mrg355_fail(MRG_E_INVALID_ARG, "request %zu: NULL pointer", i);
    if (reinterpret_cast<uintptr_t>(q.out) % esz_of(dtype))
        return mrg355_fail(MRG_E_INVALID_ARG, "request %zu: output misaligned", i);
    if (reinterpret_cast<uintptr_t>(q.streams) % 4)
        return mrg355_fail(MRG_E_INVALID_ARG, "request %zu: streams misaligned", i);
    return MRG_OK;
}

// Byte ranges [lo, hi) must not overlap.
bool disjoint(std::vector<std::pair<uintptr_t, uintptr_t>> v) {
    std::sort(v.begin(), v.end());
    for (size_t i = 1; i < v.size(); ++i)
        if (v[i].first < v[i - 1].second) return false;
    return true;
}

// Static tables of a plan, laid out as in the workspace from off_reqs on,
// into P.packed.
void pack_tables(mrg_batch_plan& P) {
    P.packed.assign(P.bytes - P.off_reqs, 0);
    char* host = P.packed.data();
    auto put = [&](size_t off, const void* src, size_t n) {
        if (n) std::memcpy(host + (off - P.off_reqs), src, n);
    };
    put(P.off_reqs, P.reqs.data(), P.reqs.size() * sizeof(BatchReq));
    put(P.off_tiles, P.tiles.data(), P.tiles.size() * sizeof(BatchTile));
    put(P.off_fin_req, P.fin_req.data(), P.fin_req.size() * sizeof(uint32_t));
    put(P.off_fin_pre, P.fin_pre.data(), P.fin_pre.size() * sizeof(uint64_t));
}

// Gang mode: within each class, tiles longest first and, among tiles of equal
// length, in (request, chunk, stream block) order, so that a gang -- G
// consecutive tiles -- holds neighbouring stream blocks of one request and
// chunk wherever the request has them; the last gang of a class is padded.
// The classes' gangs are then merged into one queue by the share of their
// class's estimated work done at each gang's midpoint, so that every class
// advances at the same pace and all of them finish together.
void order_gangs(mrg_batch_plan& P, const std::vector<double>& cost, const std::vector<uint64_t>& len) {
    const uint32_t G = P.gang;
    std::vector<uint32_t> by_cls[kClasses];
    for (uint32_t t = 0; t < P.tiles.size(); ++t)
        by_cls[batch_kind_class(static_cast<int>(P.reqs[P.tiles[t].req].kind))].push_back(t);
    struct Gang {
        double key;
        int cls;
        uint32_t first;  // index into `member`
        double cost;
        uint32_t req;    // the request of its first tile
    };
    std::vector<Gang> gangs;
    std::vector<uint32_t> member;  // tile indices, G per gang, kNoRequest for padding
    for (int c = 0; c < kClasses; ++c) {
        std::vector<uint32_t>& v = by_cls[c];
        std::stable_sort(v.begin(), v.end(), [&](uint32_t a, uint32_t b) { return len[a] > len[b]; });
        const size_t n_g = (v.size() + G - 1) / G;
        std::vector<double> gcost(n_g, 0.0);
        double total = 0.0;
        for (size_t g = 0; g < n_g; ++g) {
            for (uint32_t w = 0; w < G; ++w) {
                const size_t k = g * G + w;
                if (k < v.size()) gcost[g] = std::max(gcost[g], cost[v[k]]);
            }
            total += gcost[g];
        }
        double done = 0.0;
        for (size_t g = 0; g < n_g; ++g) {
            gangs.push_back(Gang{total > 0 ? (done + 0.5 * gcost[g]) / total : 0.0, c,
                                 static_cast<uint32_t>(member.size()), gcost[g], P.tiles[v[g * G]].req});
            done += gcost[g];
            for (uint32_t w = 0; w < G; ++w) {
                const size_t k = g * G + w;
                member.push_back(k < v.size() ? v[k] : kNoRequest);
            }
        }
    }
    std::stable_sort(gangs.begin(), gangs.end(), [](const Gang& a, const Gang& b) {
        if (a.key != b.key) return a.key < b.key;
        return a.cls < b.cls;
    });
    // Every request's gangs go to one XCD's queue (the lines its gangs share
    // are then completed in one L2): requests by estimated work, longest
    // first, each to the least loaded XCD; each queue keeps the merged order.
    std::vector<double> req_cost(P.reqs.size(), 0.0);
    for (const Gang& g : gangs) req_cost[g.req] += g.cost;
    std::vector<uint32_t> by_cost(P.reqs.size());
    for (uint32_t r = 0; r < by_cost.size(); ++r) by_cost[r] = r;
    std::stable_sort(by_cost.begin(), by_cost.end(), [&](uint32_t a, uint32_t b) { return req_cost[a] > req_cost[b]; });
    std::vector<uint8_t> xcd_of(P.reqs.size(), 0);
    double load[kXcdQueues] = {};
    for (uint32_t r : by_cost) {
        int best = 0;
        for (int x = 1; x < kXcdQueues; ++x)
            if (load[x] < load[best]) best = x;
        xcd_of[r] = static_cast<uint8_t>(best);
        load[best] += req_cost[r];
    }
    std::vector<BatchTile> out;
    out.reserve(gangs.size() * G);
    P.xq_lo[0] = 0;
    for (int x = 0; x < kXcdQueues; ++x) {
        uint32_t n = 0;
        for (const Gang& g : gangs) {
            if (xcd_of[g.req] != x) continue;
            ++n;
            for (uint32_t w = 0; w < G; ++w) {
                const uint32_t t = member[g.first + w];
                out.push_back(t == kNoRequest ? BatchTile{kNoRequest, 0, 0, 0} : P.tiles[t]);
            }
        }
        P.xq_lo[x + 1] = P.xq_lo[x] + n;
    }
    P.tiles.swap(out);
    P.n_gangs = static_cast<uint32_t>(gangs.size());
    for (int c = 0; c <= kClasses; ++c) P.tile_lo[c] = 0;
    for (int c = 0; c < kClasses; ++c) P.cls_cost[c] = 0.0;
}

// (Re)cut the plan's requests into tiles for its tile_units / wide setting.
mrg_status build(mrg_batch_plan& P) {
    P.reqs.clear();
    P.tiles.clear();
    P.fin_req.clear();
    P.fin_pre.assign(1, 0);
    std::vector<double> cost;
    std::vector<uint64_t> len;  // draw units of each tile
    // store width: automatic is one stream per lane in gang mode, where a
    // plan of such tiles runs the kernel that holds their code alone (more
    // waves fit), and the widest fitting width otherwise
    const uint32_t wide = P.wide ? P.wide : (P.gang > 1 ? 1u : 2u);
    for (size_t i = 0; i < P.user.size(); ++i) {
        const mrg_request& q = P.user[i].q;
        BatchReq R{};
        GenLaunch& L = R.L;
        L.offset = P.user[i].offset;
        L.no_writeback = P.user[i].no_writeback;
        L.streams = reinterpret_cast<uint32_t*>(q.streams);
        L.out = q.out;
        L.dist = static_cast<int>(q.dist);
        L.dtype = static_cast<int>(q.dtype);
        L.arith = kArithF64;
        L.nontemporal = 0;  // batch tiles store with ordinary stores
        L.block = kBatchBlock;
        L.param = q.dist == MRG_EXPONENTIAL ? 1.0 / q.param : 1.0;
        const int esz = static_cast<int>(esz_of(q.dtype));
        const bool plain = q.dist == MRG_UNIFORM || q.dist == MRG_RAW;
        // uniform/raw tiles store up to 16 bytes per lane (4-byte outputs: 1 or
        // 4 streams per lane), transform tiles run two streams per lane (two
        // independent chains) where the request allows
        int spl = wide == 1 ? 1 : (plain ? 16 / esz : 2);
        while (spl > 1 && (q.n_streams % spl || reinterpret_cast<uintptr_t>(q.out) % (spl * esz))) spl /= 2;
        while (spl > 1 && 64ull * spl > q.n_streams) spl /= 2;  // a wave's streams must exist
        if (plain && esz == 4 && spl == 2) spl = 1;
        if (wide == 2) {
            // a wave covers 64 * spl streams and issues its instructions for
            // all of them: keep the narrowest width that leaves the fewest
            // lanes idle in the request's last stream block (S = 300: one
            // stream per lane, 320 lane slots, rather than four, 512)
            auto slots = [&](int v) {
                const uint64_t w = 64ull * static_cast<uint64_t>(v);
                return (static_cast<uint64_t>(q.n_streams) + w - 1) / w * w;
            };
            int best = spl;
            for (int v = spl / 2; v >= 1; v /= 2)
                if (!(plain && esz == 4 && v == 2) && slots(v) < slots(best)) best = v;
            spl = best;
        }
        L.spl = spl;
        R.kind = static_cast<uint32_t>(batch_kind(L.dist, L.dtype, spl));
        if (q.n == 0) {
            P.reqs.push_back(R);
            continue;
        }
        L.S = q.n_streams;
        L.q = q.n / q.n_streams;
        L.r = static_cast<uint32_t>(q.n % q.n_streams);
        const uint64_t cnt_max = L.q + (L.r ? 1 : 0);
        const uint64_t units = L.dist == kNormal ? (cnt_max + 1) / 2 : cnt_max;
        uint64_t chunk = std::min<uint64_t>(units, P.tile_units);
        if (const uint32_t split = P.user[i].split)  // latency: spread a long request over the chip
            chunk = std::min<uint64_t>(chunk, std::max<uint64_t>(96, (units + split - 1) / split));
        const uint64_t n_chunks = (units + chunk - 1) / chunk;
        L.chunk = static_cast<uint32_t>(chunk);
        L.n_chunks = static_cast<uint32_t>(n_chunks);
        const uint64_t n_sblk = (static_cast<uint64_t>(L.S) + 64 * spl - 1) / (64 * spl);
        const uint64_t nt = n_sblk * n_chunks;
        if (P.tiles.size() + nt > 0xffffffffull) return mrg355_fail(MRG_E_INVALID_ARG, "too many tiles");
        R.n_tiles = static_cast<uint32_t>(nt);
        // chunk-major: neighbouring tiles in the queue write neighbouring
        // pieces of the same rows (4,096-request mix: 10.33 ms against 10.55 ms)
        for (uint64_t j = 0; j < n_chunks; ++j)
            for (uint64_t sb = 0; sb < n_sblk; ++sb) {
                const uint64_t u = std::min<uint64_t>(chunk, units - j * chunk);
                P.tiles.push_back(BatchTile{static_cast<uint32_t>(i), static_cast<uint32_t>(sb),
                                            static_cast<uint32_t>(j), 0});
                cost.push_back(static_cast<double>(u) * unit_cost(L.dist, L.dtype) * 64 * spl);
                len.push_back(u);
            }
        if (n_chunks > 1 && !L.no_writeback) {
            P.fin_req.push_back(static_cast<uint32_t>(i));
            P.fin_pre.push_back(P.fin_pre.back() + L.S);
        }
        P.reqs.push_back(R);
    }
    P.n_gangs = 0;
    if (P.gang > 1) {
        order_gangs(P, cost, len);
    } else {
    // grouped by class (normal, exponential, uniform/raw), longest first
    // within a class; ties keep request order
    std::vector<uint32_t> order(P.tiles.size());
    for (uint32_t i = 0; i < order.size(); ++i) order[i] = i;
    auto cls = [&](uint32_t t) { return batch_kind_class(static_cast<int>(P.reqs[P.tiles[t].req].kind)); };
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        if (cls(a) != cls(b)) return cls(a) < cls(b);
        return cost[a] > cost[b];
    });
    uint32_t n_cls[kClasses] = {0, 0, 0};
    for (int c = 0; c < kClasses; ++c) P.cls_cost[c] = 0.0;
    for (uint32_t t = 0; t < P.tiles.size(); ++t) {
        ++n_cls[cls(t)];
        P.cls_cost[cls(t)] += cost[t];
    }
    P.tile_lo[0] = 0;
    for (int c = 0; c < kClasses; ++c) P.tile_lo[c + 1] = P.tile_lo[c] + n_cls[c];
    std::vector<BatchTile> sorted(P.tiles.size());
    for (size_t i = 0; i < order.size(); ++i) sorted[i] = P.tiles[order[i]];
    P.tiles.swap(sorted);
    }
    P.fin_total = P.fin_pre.back();
    P.narrow = 1;
    for (const BatchReq& R : P.reqs) P.narrow &= batch_kind_narrow(static_cast<int>(R.kind)) ? 1u : 0u;
    // workspace layout
    const size_t n_req = P.reqs.size();
    P.off_slots = 256;
    P.off_reqs = align_up(P.off_slots + n_req * sizeof(BatchSlot), 256);
    P.off_tiles = align_up(P.off_reqs + n_req * sizeof(BatchReq), 256);
    P.off_fin_req = align_up(P.off_tiles + P.tiles.size() * sizeof(BatchTile), 256);
    P.off_fin_pre = align_up(P.off_fin_req + P.fin_req.size() * sizeof(uint32_t), 256);
    P.bytes = align_up(P.off_fin_pre + P.fin_pre.size() * sizeof(uint64_t), 256);
    pack_tables(P);
    return MRG_OK;
}

BatchLaunch launch_args(const mrg_batch_plan& P, void* ws) {
    char* base = static_cast<char*>(ws);
    BatchLaunch B{};
    B.head = reinterpret_cast<BatchHeader*>(base);
    B.slots = reinterpret_cast<BatchSlot*>(base + P.off_slots);
    B.reqs = reinterpret_cast<const BatchReq*>(base + P.off_reqs);
    B.tiles = reinterpret_cast<const BatchTile*>(base + P.off_tiles);
    B.fin_req = reinterpret_cast<const uint32_t*>(base + P.off_fin_req);
    B.fin_pre = reinterpret_cast<const uint64_t*>(base + P.off_fin_pre);
    B.n_req = static_cast<uint32_t>(P.reqs.size());
    B.n_tiles = static_cast<uint32_t>(P.tiles.size());
    B.n_fin = static_cast<uint32_t>(P.fin_req.size());
    B.fin_total = P.fin_total;
    B.n_gangs = P.n_gangs;
    B.narrow = P.narrow;
    for (int x = 0; x <= kXcdQueues; ++x) B.xq_lo[x] = P.n_gangs ? P.xq_lo[x] : 0;
    for (int c = 0; c <= kClasses; ++c) B.tile_lo[c] = P.tile_lo[c];
    return B;
}

mrg_status upload(const mrg_batch_plan& P, void* ws, hipStream_t stream) {
    hipError_t e = hipMemcpyAsync(static_cast<char*>(ws) + P.off_reqs, P.packed.data(), P.packed.size(),
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return mrg355_fail(MRG_E_HIP, "batch upload: %s", hipGetErrorString(e));
    return MRG_OK;
}

// Blocks per CU of the persistent grid: those of the requested waves per SIMD
// (4 SIMDs per CU), capped at what the kernel's registers allow at once.
uint64_t blocks_per_cu(const mrg_batch_plan& P) {
    if (P.n_gangs)
        return std::min<uint64_t>(static_cast<uint64_t>(batch_gang_blocks_per_cu(64 * P.gang, P.narrow != 0)),
                                  std::max<uint64_t>(1, 4 * P.waves_per_simd / P.gang));
    return std::min<uint64_t>(static_cast<uint64_t>(batch_blocks_per_cu()),
                              std::max<uint64_t>(1, 4 * P.waves_per_simd / (kBatchBlock / 64)));
}

mrg_status launch(const mrg_batch_plan& P, void* ws, hipStream_t stream, BatchSlot* host_slots = nullptr) {
    if (P.tiles.empty() && P.reqs.empty()) return MRG_OK;
    BatchLaunch B = launch_args(P, ws);
    B.host_slots = host_slots;
    if (P.n_gangs) {
        // one queue of gangs; the grid is what is resident at once at the
        // requested waves per SIMD, and no larger than the gang count
        const unsigned block = 64 * P.gang;
        const uint64_t per_cu = blocks_per_cu(P);
        const uint64_t grid = std::min<uint64_t>(static_cast<uint64_t>(device_cu_count()) * per_cu, P.n_gangs);
        hipError_t e = launch_batch(B, static_cast<unsigned>(grid), block, stream);
        if (e != hipSuccess) return mrg355_fail(MRG_E_HIP, "batch launch: %s", hipGetErrorString(e));
        return MRG_OK;
    }
    // The grid is at most what is resident at once, shared between the class
    // loops in proportion to the estimated work (a class with tiles gets at
    // least one block and at most one per 4 of its tiles); blocks move on to
    // the other classes when their own queue is empty.
    const uint64_t wpb = kBatchBlock / 64;
    const uint64_t per_cu = blocks_per_cu(P);
    const uint64_t total = std::max<uint64_t>(kClasses, static_cast<uint64_t>(device_cu_count()) * per_cu);
    double tot_cost = 0.0;
    for (int c = 0; c < kClasses; ++c) tot_cost += P.cls_cost[c];
    uint64_t grid = 0;
    B.block_lo[0] = 0;
    for (int c = 0; c < kClasses; ++c) {
        const uint64_t n_t = P.tile_lo[c + 1] - P.tile_lo[c];
        uint64_t nb = tot_cost > 0 ? static_cast<uint64_t>(total * (P.cls_cost[c] / tot_cost) + 0.5) : 0;
        nb = std::min<uint64_t>(std::max<uint64_t>(nb, n_t ? 1 : 0), (n_t + wpb - 1) / wpb);
        grid += nb;
        B.block_lo[c + 1] = static_cast<uint32_t>(grid);
    }
    if (grid == 0) grid = 1;  // no tiles: one block finds every queue empty
    hipError_t e = launch_batch(B, static_cast<unsigned>(grid), kBatchBlock, stream);
    if (e != hipSuccess) return mrg355_fail(MRG_E_HIP, "batch launch: %s", hipGetErrorString(e));
    return MRG_OK;
}

}  // namespace

// Workspace of mrg_batch_launch_static, for callers that cannot allocate
// device memory.  Each GPU the library runs on holds its own copy for the life
// of the process; host code reaches it only through the device address that
// hipGetSymbolAddress returns for that GPU (the array's name is a host-side
// stand-in, not a device address).
static __device__ __align__(256) char scratch[MRG_BATCH_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per GPU, looked up once

// The device address of `scratch` on the calling thread's current GPU.
mrg_status static_workspace(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return mrg355_fail(MRG_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return mrg355_fail(MRG_E_UNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return mrg355_fail(MRG_E_HIP, "static workspace address: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MRG_OK;
}

}  // namespace

namespace mrg355 {

// Plans for the serving engine: requests already validated, optionally
// starting at an offset and leaving their streams untouched.
mrg_status plan_internal(const std::vector<PlanReq>& reqs, uint32_t tile_units, mrg_batch_plan** out) {
    mrg_batch_plan* P = new (std::nothrow) mrg_batch_plan();
    if (!P) return mrg355_fail(MRG_E_NOMEM, "plan allocation failed");
    P->gen = MRG_GEN_MRG32K3A;
    P->user = reqs;
    P->tile_units = tile_units;
    P->waves_per_simd = 4;
    P->wide = 0;
    P->gang = 1;
    mrg_status st = build(*P);
    if (st) {
        delete P;
        return st;
    }
    *out = P;
    return MRG_OK;
}

size_t plan_bytes(const mrg_batch_plan* P) { return P->bytes; }
size_t plan_table_offset(const mrg_batch_plan* P) { return P->off_reqs; }
void plan_pack_tables(const mrg_batch_plan* P, char* host) {
    if (!P->packed.empty()) std::memcpy(host, P->packed.data(), P->packed.size());
}

mrg_status plan_launch(const mrg_batch_plan* P, void* ws, BatchSlot* host_slots, hipStream_t stream) {
    return launch(*P, ws, stream, host_slots);
}

}  // namespace mrg355

extern "C" {

mrg_status mrg_batch_plan_create(mrg_generator gen, const mrg_request* reqs, size_t n_req,
                                 const mrg_batch_cfg* cfg, mrg_batch_plan** plan) {
    if (gen == MRG_GEN_MRG31K3P)
        return mrg355_fail(MRG_E_UNSUPPORTED, "batched launches run MRG32k3a streams only");
    if (gen != MRG_GEN_MRG32K3A) return mrg355_fail(MRG_E_INVALID_ARG, "unknown generator id");
    if (!plan) return mrg355_fail(MRG_E_INVALID_ARG, "plan is NULL");
    if (n_req && !reqs) return mrg355_fail(MRG_E_INVALID_ARG, "reqs is NULL");
    if (n_req > 0xfffffffful) return mrg355_fail(MRG_E_INVALID_ARG, "too many requests");
    if (cfg && cfg->waves_per_simd > 16) return mrg355_fail(MRG_E_INVALID_ARG, "waves_per_simd above 16");
    if (cfg && cfg->wide_stores > 2) return mrg355_fail(MRG_E_INVALID_ARG, "wide_stores must be 0, 1 or 2");
    if (cfg && cfg->gang_waves && cfg->gang_waves != 1 && cfg->gang_waves != 2 && cfg->gang_waves != 4 &&
        cfg->gang_waves != 8)
        return mrg355_fail(MRG_E_INVALID_ARG, "gang_waves must be 0, 1, 2, 4 or 8");
    std::vector<std::pair<uintptr_t, uintptr_t>> sr, orng;
    for (size_t i = 0; i < n_req; ++i) {
        if (mrg_status st = validate_request(reqs[i], i)) return st;
        if (reqs[i].n == 0) continue;
        uintptr_t s0 = reinterpret_cast<uintptr_t>(reqs[i].streams);
        uintptr_t o0 = reinterpret_cast<uintptr_t>(reqs[i].out);
        sr.emplace_back(s0, s0 + static_cast<uintptr_t>(reqs[i].n_streams) * sizeof(mrg_stream));
        orng.emplace_back(o0, o0 + static_cast<uintptr_t>(reqs[i].n) * esz_of(reqs[i].dtype));
    }
    if (!disjoint(sr)) return mrg355_fail(MRG_E_INVALID_ARG, "requests share stream records");
    if (!disjoint(orng)) return mrg355_fail(MRG_E_INVALID_ARG, "requests share output bytes");
    mrg_batch_plan* P = new (std::nothrow) mrg_batch_plan();
    if (!P) return mrg355_fail(MRG_E_NOMEM, "plan allocation failed");
    P->gen = gen;
    P->user.resize(n_req);
    for (size_t i = 0; i < n_req; ++i) P->user[i] = PlanReq{reqs[i], 0, 0};
    P->tile_units = (cfg && cfg->tile_units) ? cfg->tile_units : kDefaultTileUnits;
    P->waves_per_simd = (cfg && cfg->waves_per_simd) ? cfg->waves_per_simd : kDefaultWavesPerSimd;
    P->wide = cfg ? cfg->wide_stores : 0;
    P->gang = (cfg && cfg->gang_waves) ? cfg->gang_waves : kDefaultGang;
    mrg_status st = build(*P);
    if (st) {
        delete P;
        return st;
    }
    *plan = P;
    return MRG_OK;
}

void mrg_batch_plan_destroy(mrg_batch_plan* plan) { delete plan; }

mrg_status mrg_batch_workspace_size(const mrg_batch_plan* plan, size_t* bytes) {
    if (!plan || !bytes) return mrg355_fail(MRG_E_INVALID_ARG, "NULL plan or bytes");
    *bytes = plan->bytes;
    return MRG_OK;
}

// Shapes the autotuner times: tile length (draw units per wave tile) x block
// shape (class queues of single waves, or gangs of 4 or 8 waves) x streams per
// lane (widest stores a request allows, or one stream per lane) x waves per
// SIMD.  Tile length sets the per-stream work-item count (a stream of u units
// is cut into ceil(u / tile_units) work-items).
static constexpr uint32_t kTuneTileUnits[] = {192, 256, 512, 1024, 2048, 4096, 8192};
static constexpr uint32_t kTuneGang[] = {1, 4, 8};
static constexpr uint32_t kTuneWide[] = {1, 2};
static constexpr uint32_t kTuneWaves[] = {2, 3, 4, 5, 6};

mrg_status mrg_batch_autotune_workspace_size(const mrg_batch_plan* plan, size_t* bytes) {
    if (!plan || !bytes) return mrg355_fail(MRG_E_INVALID_ARG, "NULL plan or bytes");
    size_t most = plan->bytes;
    for (uint32_t tu : kTuneTileUnits)
        for (uint32_t g : kTuneGang)
            for (uint32_t w : kTuneWide) {
                mrg_batch_plan trial = *plan;
                trial.tile_units = tu;
                trial.gang = g;
                trial.wide = w;
                if (mrg_status st = build(trial)) return st;
                most = std::max(most, trial.bytes);
            }
    *bytes = most;
    return MRG_OK;
}

mrg_status mrg_batch_tile_count(const mrg_batch_plan* plan, size_t* tiles) {
    if (!plan || !tiles) return mrg355_fail(MRG_E_INVALID_ARG, "NULL plan or tiles");
    *tiles = plan->tiles.size();
    return MRG_OK;
}

mrg_status mrg_batch_upload(const mrg_batch_plan* plan, void* dev_workspace, hipStream_t stream) {
    if (!plan || !dev_workspace) return mrg355_fail(MRG_E_INVALID_ARG, "NULL plan or workspace");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % 256)
        return mrg355_fail(MRG_E_INVALID_ARG, "workspace must be 256-byte aligned");
    return upload(*plan, dev_workspace, stream);
}

mrg_status mrg_batch_launch(const mrg_batch_plan* plan, void* dev_workspace, hipStream_t stream) {
    if (!plan || !dev_workspace) return mrg355_fail(MRG_E_INVALID_ARG, "NULL plan or workspace");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % 256)
        return mrg355_fail(MRG_E_INVALID_ARG, "workspace must be 256-byte aligned");
    return launch(*plan, dev_workspace, stream);
}

mrg_status mrg_batch_launch_static(const mrg_batch_plan* plan, hipStream_t stream) {
    if (!plan) return mrg355_fail(MRG_E_INVALID_ARG, "NULL plan");
    if (plan->bytes > MRG_BATCH_STATIC_WORKSPACE_BYTES)
        return mrg355_fail(MRG_E_NOMEM,
                           "the plan needs %zu bytes of workspace, the static workspace holds %zu: "
                           "use mrg_batch_launch with a workspace of its own",
                           plan->bytes, static_cast<size_t>(MRG_BATCH_STATIC_WORKSPACE_BYTES));
    void* ws = nullptr;
    if (mrg_status st = static_workspace(&ws)) return st;
    if (!plan->packed.empty()) {
        hipError_t e = hipMemcpyAsync(static_cast<char*>(ws) + plan->off_reqs, plan->packed.data(),
                                      plan->packed.size(), hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return mrg355_fail(MRG_E_HIP, "static batch upload: %s", hipGetErrorString(e));
    }
    return launch(*plan, ws, stream);
}

mrg_status mrg_batch_request_times(const mrg_batch_plan* plan, const void* dev_workspace,
                                   uint64_t* host_ticks, hipStream_t stream) {
    if (!plan || !dev_workspace || !host_ticks) return mrg355_fail(MRG_E_INVALID_ARG, "NULL argument");
    const size_t n = plan->reqs.size();
    std::vector<BatchSlot> slots(n);
    BatchHeader head{};
    const char* base = static_cast<const char*>(dev_workspace);
    hipError_t e = hipMemcpyAsync(&head, base, sizeof(head), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess && n)
        e = hipMemcpyAsync(slots.data(), base + plan->off_slots, n * sizeof(BatchSlot), hipMemcpyDeviceToHost,
                           stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return mrg355_fail(MRG_E_HIP, "request times: %s", hipGetErrorString(e));
    host_ticks[0] = head.t_start;
    for (size_t i = 0; i < n; ++i) host_ticks[1 + i] = slots[i].done ? slots[i].t_done : 0;
    return MRG_OK;
}

mrg_status mrg_batch_autotune(mrg_batch_plan* plan, void* dev_workspace, size_t workspace_bytes,
                              hipStream_t stream, mrg_batch_cfg* best, double* best_ms) {
    if (!plan || !dev_workspace) return mrg355_fail(MRG_E_INVALID_ARG, "NULL plan or workspace");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % 256)
        return mrg355_fail(MRG_E_INVALID_ARG, "workspace must be 256-byte aligned");
    // save every request's stream records
    std::vector<std::vector<char>> saved(plan->user.size());
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < plan->user.size() && e == hipSuccess; ++i) {
        const mrg_request& q = plan->user[i].q;
        if (!q.n) continue;
        saved[i].resize(static_cast<size_t>(q.n_streams) * sizeof(mrg_stream));
        e = hipMemcpyAsync(saved[i].data(), q.streams, saved[i].size(), hipMemcpyDeviceToHost, stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return mrg355_fail(MRG_E_HIP, "autotune save: %s", hipGetErrorString(e));

    const uint32_t orig_tu = plan->tile_units, orig_w = plan->waves_per_simd, orig_g = plan->gang,
                   orig_wide = plan->wide;
    double best_t = 1e30;
    uint32_t best_tu = orig_tu, best_w = orig_w, best_g = orig_g, best_wide = orig_wide;
    hipEvent_t a = nullptr, b = nullptr;
    e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    mrg_status st = MRG_OK;
    for (uint32_t tu : kTuneTileUnits)
        for (uint32_t g : kTuneGang)
            for (uint32_t wide : kTuneWide) {
                if (st || e != hipSuccess) break;
                plan->tile_units = tu;
                plan->gang = g;
                plan->wide = wide;
                if ((st = build(*plan))) break;
                if (plan->bytes > workspace_bytes) continue;  // does not fit the caller's workspace
                if ((st = upload(*plan, dev_workspace, stream))) break;
                uint64_t timed_per_cu = 0;
                for (uint32_t w : kTuneWaves) {
                    plan->waves_per_simd = w;
                    // a waves setting the kernel's registers cap to the
                    // grid of the previous one is not timed again
                    const uint64_t per_cu = blocks_per_cu(*plan);
                    if (per_cu == timed_per_cu) continue;
                    timed_per_cu = per_cu;
                    if ((st = launch(*plan, dev_workspace, stream))) break;  // warm-up
                    e = hipEventRecord(a, stream);
                    for (int rep = 0; rep < 3 && !st; ++rep) st = launch(*plan, dev_workspace, stream);
                    if (e == hipSuccess) e = hipEventRecord(b, stream);
                    if (e == hipSuccess) e = hipEventSynchronize(b);
                    float ms = 0;
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
                    if (st || e != hipSuccess) break;
                    if (ms / 3 < best_t) {
                        best_t = ms / 3;
                        best_tu = tu;
                        best_w = w;
                        best_g = g;
                        best_wide = wide;
                    }
                }
            }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    // restore the streams, keep the best shape
    for (size_t i = 0; i < plan->user.size() && e == hipSuccess; ++i) {
        if (saved[i].empty()) continue;
        e = hipMemcpyAsync(plan->user[i].q.streams, saved[i].data(), saved[i].size(), hipMemcpyHostToDevice,
                           stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    const bool found = best_t < 1e30;
    plan->tile_units = found ? best_tu : orig_tu;
    plan->waves_per_simd = found ? best_w : orig_w;
    plan->gang = found ? best_g : orig_g;
    plan->wide = found ? best_wide : orig_wide;
    mrg_status st2 = build(*plan);
    if (st) return st;
    if (e != hipSuccess) return mrg355_fail(MRG_E_HIP, "autotune: %s", hipGetErrorString(e));
    if (st2) return st2;
    if (plan->bytes <= workspace_bytes)
        if ((st2 = upload(*plan, dev_workspace, stream))) return st2;
    if (best) {
        best->tile_units = plan->tile_units;
        best->waves_per_simd = plan->waves_per_simd;
        best->wide_stores = plan->wide;
        best->gang_waves = plan->gang;
    }
    if (best_ms) *best_ms = best_t < 1e30 ? best_t : 0.0;
    return MRG_OK;
}

}  // extern "C"
