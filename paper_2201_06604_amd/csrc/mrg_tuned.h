// mrg_tuned.h -- launch shapes of mrg_generate's automatic plan, per output
// kind and size class.  Results never depend on them: every value is a
// function of (stream, draw index) only.
//
// Written by `python -m paper_2201_06604_amd.tune_plain --write` from timings
// on MI355X (the tuner times candidate shapes on a representative workload of
// each class and keeps the fastest; its docstring lists them).
#pragma once

#include <stdint.h>

namespace mrg355 {

struct TunedShape {
    uint16_t spl;        // streams per lane asked for (then narrowed to what the shape allows)
    uint16_t block;      // threads per block
    uint16_t waves;      // waves the grid aims at (sets the chunk)
    uint16_t min_units;  // shortest chunk, draw units
    uint16_t lock;       // 1 = lockstep rows once the grid has two waves per SIMD
    uint16_t xcd;        // 1 = XCD-contiguous block order
};

// Kinds: uniform f64, uniform f32, raw u32, normal f64, normal f32,
// exponential f64, exponential f32.  Size classes by the call's draw count n:
// below 2^18, 2^22, 2^26, 2^29, and above (timed at 2^16, 2^20, 2^24, 2^28
// and 2^30 draws: 256 x 256, 1,024 x 1,024, 16,384 x 1,024, 65,536 x 4,096
// and 262,144 x 4,096 streams x draws).
constexpr int kTunedKinds = 7;
constexpr int kTunedClasses = 5;
// clang-format off
constexpr TunedShape kTuned[kTunedKinds][kTunedClasses] = {
    {{1, 256, 2048, 32, 0, 1}, {1, 256, 2048, 32, 0, 1}, {1, 512, 2048, 32, 1, 1}, {2, 512, 2048, 96, 1, 1}, {2, 512, 2048, 96, 1, 1}},
    {{1, 512, 4096, 32, 0, 0}, {1, 512, 4096, 32, 0, 0}, {1, 512, 4096, 32, 0, 0}, {4, 512, 4096, 96, 0, 0}, {4, 512, 4096, 96, 0, 0}},
    {{1, 512, 4096, 32, 0, 0}, {1, 512, 4096, 32, 0, 0}, {1, 512, 4096, 32, 0, 0}, {4, 512, 4096, 96, 0, 0}, {4, 512, 4096, 96, 0, 0}},
    {{1, 256, 8192, 32, 0, 1}, {1, 256, 8192, 32, 0, 1}, {1, 256, 8192, 32, 0, 1}, {2, 256, 8192, 96, 0, 1}, {2, 256, 8192, 96, 0, 1}},
    {{1, 256, 8192, 32, 0, 1}, {1, 256, 8192, 32, 0, 1}, {1, 256, 8192, 32, 0, 1}, {2, 256, 8192, 96, 0, 1}, {2, 256, 8192, 96, 0, 1}},
    {{1, 256, 4096, 32, 0, 1}, {1, 256, 4096, 32, 0, 1}, {1, 256, 4096, 32, 0, 1}, {2, 256, 4096, 96, 0, 1}, {2, 256, 4096, 96, 0, 1}},
    {{1, 256, 4096, 32, 0, 1}, {1, 256, 4096, 32, 0, 1}, {1, 256, 4096, 32, 0, 1}, {2, 256, 4096, 96, 0, 1}, {2, 256, 4096, 96, 0, 1}},
};
// clang-format on

}  // namespace mrg355
