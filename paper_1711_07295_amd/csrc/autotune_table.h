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
constexpr double kFilterNsPerPair[6] = {2.9672e-05, 4.8339e-05, 1.1220e-04, 8.5153e-04, 2.0138e-03, 5.7949e-03};
constexpr double kSlowEntryNs = 3.7727e+00;
constexpr double kSurvivorNs = 7.7342e-02;
constexpr double kSurvivorWaveNs[6] = {4.6449e+00, 4.5711e+00, 4.6161e+00, 5.6737e+00, 6.9138e+00, 1.7046e+01};
constexpr double kPairsPerStep[6] = {6144.0, 3072.0, 3072.0, 64.0, 64.0, 64.0};
constexpr double kClassLaunchNs[6] = {4.0354e+04, 3.1596e+04, 4.0835e+04, 3.5796e+04, 4.2994e+04, 7.3710e+04};
constexpr uint32_t kClassTileCols[6] = {4096, 4096, 4096, 2048, 1024, 2048};
}  // namespace ssj
