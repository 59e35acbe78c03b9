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
// Timings of the tuning run that wrote this table (MI355X, median of 7 launches):
// uniform f64, 256 x 256: 21.6 us (entry before: 22.4 us; 12 shapes timed)
// uniform f32, 256 x 256: 21.4 us (entry before: 22.1 us; 12 shapes timed)
// raw u32, 256 x 256: 21.4 us (entry before: 22.9 us; 12 shapes timed)
// normal f64, 256 x 256: 26.1 us (entry before: 26.1 us; 8 shapes timed)
// normal f32, 256 x 256: 24.6 us (entry before: 25.3 us; 8 shapes timed)
// exponential f64, 256 x 256: 23.4 us (entry before: 23.4 us; 12 shapes timed)
// exponential f32, 256 x 256: 22.6 us (entry before: 23.3 us; 12 shapes timed)
// uniform f64, 1024 x 1024: 23.3 us (entry before: 24.4 us; 12 shapes timed)
// uniform f32, 1024 x 1024: 23.6 us (entry before: 25.4 us; 12 shapes timed)
// raw u32, 1024 x 1024: 23.7 us (entry before: 25.7 us; 12 shapes timed)
// normal f64, 1024 x 1024: 29.2 us (entry before: 29.2 us; 13 shapes timed)
// normal f32, 1024 x 1024: 27.3 us (entry before: 27.3 us; 13 shapes timed)
// exponential f64, 1024 x 1024: 26.3 us (entry before: 26.3 us; 12 shapes timed)
// exponential f32, 1024 x 1024: 25.8 us (entry before: 25.8 us; 12 shapes timed)
// uniform f64, 16384 x 1024: 38.1 us (entry before: 41.0 us; 60 shapes timed)
// uniform f32, 16384 x 1024: 32.6 us (entry before: 35.9 us; 32 shapes timed)
// raw u32, 16384 x 1024: 33.2 us (entry before: 35.8 us; 32 shapes timed)
// normal f64, 16384 x 1024: 49.8 us (entry before: 54.9 us; 28 shapes timed)
// normal f32, 16384 x 1024: 44.5 us (entry before: 48.1 us; 28 shapes timed)
// exponential f64, 16384 x 1024: 48.4 us (entry before: 51.5 us; 36 shapes timed)
// exponential f32, 16384 x 1024: 43.4 us (entry before: 45.7 us; 36 shapes timed)
// uniform f64, 65536 x 4096: 363.8 us (entry before: 371.9 us; 72 shapes timed)
// uniform f32, 65536 x 4096: 187.5 us (entry before: 214.3 us; 44 shapes timed)
// raw u32, 65536 x 4096: 184.8 us (entry before: 236.0 us; 44 shapes timed)
// normal f64, 65536 x 4096: 519.1 us (entry before: 533.2 us; 44 shapes timed)
// normal f32, 65536 x 4096: 375.5 us (entry before: 409.3 us; 44 shapes timed)
// exponential f64, 65536 x 4096: 474.2 us (entry before: 497.0 us; 40 shapes timed)
// exponential f32, 65536 x 4096: 338.6 us (entry before: 381.5 us; 40 shapes timed)
// uniform f64, 262144 x 4096: 1344.7 us (entry before: 1344.7 us; 56 shapes timed)
// uniform f32, 262144 x 4096: 750.9 us (entry before: 781.3 us; 32 shapes timed)
// raw u32, 262144 x 4096: 733.1 us (entry before: 816.0 us; 32 shapes timed)
// normal f64, 262144 x 4096: 2084.8 us (entry before: 2084.8 us; 28 shapes timed)
// normal f32, 262144 x 4096: 1508.9 us (entry before: 1581.9 us; 28 shapes timed)
// exponential f64, 262144 x 4096: 1915.8 us (entry before: 1915.8 us; 28 shapes timed)
// exponential f32, 262144 x 4096: 1359.3 us (entry before: 1389.1 us; 28 shapes timed)
// clang-format off
constexpr TunedShape kTuned[kTunedKinds][kTunedClasses] = {
    {{1, 256, 1024, 32, 0, 0}, {1, 256, 1024, 32, 0, 0}, {1, 256, 4096, 32, 0, 0}, {1, 512, 2048, 32, 1, 0}, {2, 512, 2048, 96, 1, 1}},  // uniform f64
    {{1, 256, 1024, 32, 0, 1}, {1, 256, 1024, 32, 0, 1}, {1, 512, 2048, 32, 0, 0}, {1, 256, 16384, 32, 0, 0}, {4, 256, 4096, 32, 0, 0}},  // uniform f32
    {{1, 256, 1024, 32, 0, 0}, {1, 256, 1024, 32, 0, 0}, {1, 512, 2048, 32, 0, 0}, {1, 256, 8192, 32, 0, 0}, {4, 256, 8192, 32, 0, 0}},  // raw u32
    {{1, 256, 8192, 32, 0, 1}, {1, 256, 8192, 32, 0, 1}, {1, 512, 2048, 32, 0, 1}, {1, 256, 8192, 32, 0, 0}, {2, 256, 8192, 96, 0, 1}},  // normal f64
    {{1, 512, 1024, 32, 0, 0}, {1, 256, 8192, 32, 0, 1}, {1, 256, 2048, 32, 0, 0}, {1, 256, 8192, 32, 0, 0}, {1, 512, 16384, 32, 0, 0}},  // normal f32
    {{1, 256, 4096, 32, 0, 1}, {1, 256, 4096, 32, 0, 1}, {1, 512, 2048, 32, 0, 1}, {2, 256, 8192, 32, 0, 0}, {2, 256, 4096, 96, 0, 1}},  // exponential f64
    {{1, 512, 1024, 32, 0, 0}, {1, 256, 4096, 32, 0, 1}, {1, 256, 2048, 32, 0, 0}, {2, 256, 2048, 32, 0, 0}, {2, 512, 4096, 32, 0, 1}},  // exponential f32
};
// clang-format on

}  // namespace mrg355
