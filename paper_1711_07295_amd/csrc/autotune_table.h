// Costs the width autotuner weighs, measured by
// paper_1711_07295_amd/calibrate.py on subsets of the 1,000,000-set
// self-join workload at Jaccard 4/5 (fixed widths).
// Device: AMD Radeon Graphics (gfx950:sramecc+:xnack-, 256 CUs); 2026-12-03.
// Per width b = 64, 128, 256, 512: filter kernel ns per band pair (sets of
// 2..40 tokens); ns of a class launch that does not grow with its work (4,000
// sets); the tile width (columns) with the shortest filter time.  And ns per
// false survivor (the filter's slow path and queue writes, and its
// verification; from the sets of 50..89 tokens at b = 64 against b = 128).
#pragma once
#include <cstdint>

namespace ssj {
constexpr double kFilterNsPerPair[4] = {3.1104e-05, 4.7709e-05, 1.1181e-04, 8.5296e-04};
constexpr double kSurvivorNs = 3.7810e+00;
constexpr double kClassLaunchNs[4] = {3.3195e+04, 3.1676e+04, 4.1395e+04, 3.6435e+04};
constexpr uint32_t kClassTileCols[4] = {4096, 4096, 4096, 2048};
}  // namespace ssj
