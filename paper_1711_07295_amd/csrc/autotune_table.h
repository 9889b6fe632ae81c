// Costs the width autotuner weighs, measured by
// paper_1711_07295_amd/calibrate.py on subsets of the 1,000,000-set
// self-join workload at Jaccard 4/5 (fixed widths).
// Device: AMD Radeon Graphics (gfx950:sramecc+:xnack-, 256 CUs); 2026-12-03.
// Per width b = 64 .. 2048: filter kernel ns per band pair (sets of 2..40
// tokens); ns of a class launch that does not grow with its work (4,000
// sets); the tile width (columns) with the shortest filter time; the pairs
// of one step of the width's kernel.  And the ns of a slow-path entry and the
// ns a survivor adds (queue writes, verification), from the sets of 50..89
// tokens (64 against 128 bits at 4/5; 64 bits at 1/2); per width, the ns one
// wave takes to stage a survivor, from one tile where nearly every pair
// survives (64 x 2048 random sets of b tokens at 1/2).
#pragma once
#include <cstdint>

namespace ssj {
constexpr double kFilterNsPerPair[6] = {2.9462e-05, 4.2423e-05, 7.9398e-05, 2.1332e-04, 8.6747e-04, 5.7976e-03};
constexpr double kSlowEntryNs = 3.6491e+00;
constexpr double kSurvivorNs = 7.7376e-02;
constexpr double kSurvivorWaveNs[6] = {4.5648e+00, 4.4890e+00, 4.5477e+00, 5.1089e+00, 5.3780e+00, 1.6892e+01};
constexpr double kPairsPerStep[6] = {6144.0, 4096.0, 5120.0, 4096.0, 2048.0, 64.0};
constexpr double kClassLaunchNs[6] = {4.1035e+04, 3.5716e+04, 4.1474e+04, 3.5595e+04, 4.2834e+04, 7.3631e+04};
constexpr uint32_t kClassTileCols[6] = {4096, 4096, 4096, 4096, 4096, 2048};
}  // namespace ssj
