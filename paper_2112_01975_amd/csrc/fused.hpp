// fused.hpp -- launch interface of the single-pass D3Q27 step (z-march).
#pragma once

#include <vector>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace lbm {

struct FusedGrid {
    int tx, ty, tz;        // tile width in x, height in y, planes per z-chunk
    int zb, ze;            // the launch collides planes [zb, ze), in chunks of tz from zb
    int ntx, nty, nzc;     // tiles in x, y and z-chunks
    int items;             // ntx * nty * nzc work items
    int item0, count;      // this launch runs items [item0, item0 + count)
    int per_xcd;           // items per XCD (ceil(count / 8))
    int blocks;            // launched workgroups = 8 * per_xcd
    double *partials;      // nullable: item i writes the FP64 totals (mass, momentum, domain
                           // count; kPartialSlots values) of the nodes it collides, as pulled
                           // from the input state, into row slot0 + i
    int slot0;
};

FusedGrid fused_grid(const Geom &g, int tx, int ty, int tz, int zb, int ze);

// The launches of one grid: windows of at most `window` consecutive items, so that each
// round of work items starts together (neighbouring tiles then march in step and share
// their halo lines in L2, which later rounds of one launch, started as earlier items
// finish, do not).
std::vector<FusedGrid> fused_windows(const FusedGrid &fg, int window);

// Solid geometry for the fused step (nullptr without solid nodes):
//   links[n]  per-node solid-neighbour bits from fused_links;
//   pflags[z] bit 0: plane z has a solid node, bit 1: planes z-1..z+1 have one;
//   qlo[n]    with interpolated walls only: bit i when the wall link crossed by
//             population i has q < 1/2 (fused_qlo).
struct FusedMask {
    const uint32_t *links;
    const uint32_t *pflags;
    const uint32_t *qlo;
};

using FusedLaunch = void (*)(hipStream_t, const void *A, void *B, const Geom &, const FusedMask &,
                             const void *params, const FusedGrid &);

// One launch of a fused step: the kernel and the plane range it collides. A step is a
// list of these over disjoint ranges that cover every plane: runs of planes within three
// planes of a solid node take the masked kernel, the others the unmasked one (whose
// registers are not shared with the bounce-back code).
struct FusedSeg {
    FusedLaunch fn;
    FusedGrid fg;
};

// bit i of links[n]: the source node n - c_i of population i is solid; bit 27: n is solid
void fused_links(hipStream_t s, const uint8_t *mask, uint32_t *links, const Geom &g);

// the q < 1/2 bits from the links and the device wall fractions ([Q][qs], compute precision)
void fused_qlo(hipStream_t s, const uint32_t *links, const void *lq, bool fp64, uint32_t *qlo, const Geom &g);

// nullptr when no fused variant exists for this combination
// lat: how the kernel addresses a lattice: 0 one buffer resource (below 4 GiB), 1 two
// buffer resources (populations 0-13 and 14-26, each below 4 GiB), 2 one resource per
// group of four (FP32) or two (FP64) populations (population arrays below 1 GiB or 2 GiB);
// interp: walls with per-link fractions (Params::link_q), interpolated bounce-back
FusedLaunch fused_launcher(bool fp64, bool masked, int tx, int ty, int lat, bool interp);

}  // namespace lbm
