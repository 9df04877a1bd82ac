// fused.hpp -- launch interface of the single-pass D3Q27 step (z-march).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace lbm {

struct FusedGrid {
    int ty, tz;            // tile height in y, planes per z-chunk
    int ntx, nty, nzc;     // tiles in x, y and z-chunks
    int items;             // ntx * nty * nzc work items
    int per_xcd;           // items per XCD (ceil(items / 8))
    int blocks;            // launched workgroups = 8 * per_xcd
};

FusedGrid fused_grid(const Geom &g, int ty, int tz);

using FusedLaunch = void (*)(hipStream_t, const void *A, void *B, const Geom &, const uint8_t *mask,
                             const void *params, const FusedGrid &);

// nullptr when no fused variant exists for this combination
FusedLaunch fused_launcher(bool fp64, bool masked, int ty);

}  // namespace lbm
