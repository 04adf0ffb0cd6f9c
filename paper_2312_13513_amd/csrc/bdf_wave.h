// Wave-per-cell and tile (16 lanes per cell) integrators (bdf_wave.hip):
// tables and launcher.
#pragma once

#include "chem_internal.h"

namespace chem {

// For each species k, the reactions with a non-zero net coefficient, in
// increasing reaction order: entries inc[inc_off[k] .. inc_off[k+1]) hold
// (reaction index, net coefficient).
struct WaveTables {
    const int *inc_off;
    const int2 *inc;
};

// Padded row count of the wave kernel for N unknowns (0 = unsupported).
int wave_kernel_rows(int N);

// Whether the wave (lanes = 64) or tile (lanes = 16) kernel of this mechanism
// keeps its reaction scratch (7 R doubles per cell in flight) in global memory
// because it does not fit in LDS.
bool wave_uses_global_scratch(const DevMechView &m, int lanes);

// lanes = 64: one wave per cell (N <= 64); lanes = 16: four cells per wave
// (N <= 16).  qscratch holds max_groups slices of 7 R doubles, used when the
// reaction scratch does not fit in LDS
// (wave_uses_global_scratch); the launch then runs at most max_groups groups.
hipError_t launch_bdf_wave(const DevMechView &m, const WaveTables &wt, double *T, const double *p,
                           double *Y, int64_t ldY, int64_t n, double dt, const BdfParams &prm,
                           int32_t *status, int32_t *counters, unsigned long long *queue,
                           double *qscratch, int max_groups, bool fp32_lu, int lanes, hipStream_t s);

}  // namespace chem
