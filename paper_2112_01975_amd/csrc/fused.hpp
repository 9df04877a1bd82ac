// fused.hpp -- launch interface of the single-pass D3Q27 step (z-march).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace lbm {

struct FusedGrid {
    int tx, ty, tz;        // tile width in x, height in y, planes per z-chunk
    int ntx, nty, nzc;     // tiles in x, y and z-chunks
    int items;             // ntx * nty * nzc work items
    int per_xcd;           // items per XCD (ceil(items / 8))
    int blocks;            // launched workgroups = 8 * per_xcd
    unsigned pop_bytes;    // Q * qs * sizeof(S): extent of one population lattice (< 4 GiB)
};

FusedGrid fused_grid(const Geom &g, int tx, int ty, int tz);

using FusedLaunch = void (*)(hipStream_t, const void *A, void *B, const Geom &, const uint8_t *mask,
                             const void *params, const FusedGrid &);

// nullptr when no fused variant exists for this combination
FusedLaunch fused_launcher(bool fp64, bool masked, int tx, int ty);

}  // namespace lbm
