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
constexpr double kFilterNsPerPair[6] = {2.9350e-05, 4.7487e-05, 1.1156e-04, 2.1471e-04, 8.6554e-04, 5.8077e-03};
constexpr double kSlowEntryNs = 3.9069e+00;
constexpr double kSurvivorNs = 7.7485e-02;
constexpr double kSurvivorWaveNs[6] = {4.6819e+00, 4.5574e+00, 4.6085e+00, 5.2081e+00, 5.5160e+00, 1.6888e+01};
constexpr double kPairsPerStep[6] = {6144.0, 3072.0, 3072.0, 4096.0, 2048.0, 64.0};
constexpr double kClassLaunchNs[6] = {4.0475e+04, 3.1196e+04, 4.1075e+04, 3.5995e+04, 4.2435e+04, 7.4510e+04};
constexpr uint32_t kClassTileCols[6] = {4096, 4096, 4096, 4096, 4096, 2048};
}  // namespace ssj
