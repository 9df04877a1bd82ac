// runtime.hip -- C ABI of the single-simulation path: parameter validation,
// device memory, the step loop, the FP64 watchdog, moments output, checkpoints.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbm2p.h"
#include "fused.hpp"
#include "kernels.hpp"
#include "runtime_common.hpp"
#include "thermo_host.hpp"

using namespace lbm;

// Device scratch of lbm_moments_noalloc: the moment pass's partial rows followed by the
// intermediate rows of the FP64 reduction tree. Every device the library runs on holds one
// copy until the process ends. Host code never passes this name to a kernel or a copy: it
// uses the address that hipGetSymbolAddress returns for the device (device_scratch below).
constexpr size_t kScratchBytes = size_t(8) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

struct lbm_ctx {
    lbm_params p;
    int D = 0, Q = 0;
    bool fp64 = true, masked = false;
    Geom g{};
    int device = 0;
    size_t sbytes = 8;               // bytes per stored population
    hipStream_t own = nullptr, stream = nullptr;
    void *A = nullptr, *B = nullptr; // population lattices
    void *rho = nullptr, *gfl = nullptr;
    uint8_t *mask = nullptr;
    uint32_t *links = nullptr;       // solid-neighbour bits for the fused step (masked only)
    uint32_t *pflags = nullptr;      // per-plane solid flags for the fused step (masked only)
    uint32_t *qlo = nullptr;         // q < 1/2 bits of the wall links for the fused step (link_q only)
    void *wall = nullptr;            // per-node wall densities in compute precision (optional)
    void *lq = nullptr;              // per-link wall fractions in compute precision (optional)
    double *partials = nullptr;
    double *fpart = nullptr;         // fused step: one row of FP64 totals per work item
    int nfslots = 0;                 // rows of fpart
    bool fold = false;               // the fused step accumulates the totals (FP32, no mask)
    bool folded = false;             // fpart holds the totals of the state that entered the last step
    double *htot = nullptr;          // mapped pinned host memory: the reduction tree's result
    double *htot_dev = nullptr;      // its device address
    int64_t steps = 0;               // steps since the last lbm_init_fields / lbm_set_populations
    double last[5] = {0, 0, 0, 0, 0};  // the latest watchdog check: M, J, domain count
    int64_t last_step = -1;          // the step index of the state those totals describe
    double *rscratch = nullptr;      // intermediate rows of the reduction tree
    double *scratch = nullptr;       // this device's static scratch (lbm_moments_noalloc), not owned
    double *io = nullptr;            // FP64 staging for init / output: (1 + D) * N
    double *ptens = nullptr;         // FP64 pressure tensor output, D(D+1)/2 * N (on first use)
    void *pack = nullptr;            // contiguous staging of one field for padded rows (on first use)
    int nblk = 0;
    Params<double> pd{};
    Params<float> pf{};
    KernelSet ks{};
    hipGraphExec_t gexec = nullptr;  // steps off the fused kernel: kGraphSteps captured once, replayed
    void *gA = nullptr;              // the lattice those captured steps start from
    bool use_graph = false;
    bool single = false;             // D2Q9: single-pass step (ks.single) instead of moments + collide
    FusedLaunch fused = nullptr;     // single-pass step when available (D3Q27): the first segment's kernel
    std::vector<FusedSeg> segs;      // the launches of one fused step, over disjoint plane ranges
    bool initialized = false;
    int sticky = 0;
    double M0 = 0.0;
    std::string err;
};

namespace {

thread_local std::string g_create_err;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_addr[kMaxDevices] = {};

// Address of the static scratch on device dev, which must be current: resolved on the first
// request for that device, then kept (each device holds its own copy at its own address).
hipError_t device_scratch(int dev, double **out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_addr[dev] = (double *)p;
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

int fail(lbm_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg; else g_create_err = msg;
    return code;
}

#define HIP_OR_FAIL(c, call)                                                                  \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail((c), LBM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

const void *params_ptr(const lbm_ctx *c) { return c->fp64 ? (const void *)&c->pd : (const void *)&c->pf; }

void free_ctx(lbm_ctx *c) {
    if (!c) return;
    void *ptrs[] = {c->A, c->B, c->rho, c->gfl, c->mask, c->links, c->pflags, c->qlo, c->wall, c->lq, c->partials,
                    c->io, c->ptens, c->pack, c->fpart, c->rscratch};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    if (c->htot) (void)hipHostFree(c->htot);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->own) (void)hipStreamDestroy(c->own);
    delete c;
}

// reduction tree over partial rows -> host[5] (synchronous): the last level writes the
// totals straight into mapped pinned host memory, so a check is the tree and a stream sync
int reduce_rows(lbm_ctx *c, const double *rows, int n, double host[5]) {
    launch_reduce(c->stream, rows, n, c->rscratch, c->htot_dev);
    HIP_OR_FAIL(c, hipGetLastError());
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < 5; ++k) host[k] = c->htot[k];
    return LBM_OK;
}

// mass/momentum of the current state -> host[5]; also the domain-error count
int reduce_state(lbm_ctx *c, double host[5]) {
    c->ks.moments(c->stream, c->A, c->g, c->mask, params_ptr(c), c->rho, c->gfl, c->partials);
    return reduce_rows(c, c->partials, c->nblk, host);
}

// Watchdog check. After a single-pass step it reduces the rows that step wrote while pulling
// its input state (no moment pass); otherwise it runs the moment pass on the current state.
int watchdog(lbm_ctx *c) {
    double t[5];
    int rc = c->folded ? reduce_rows(c, c->fpart, c->nfslots, t) : reduce_state(c, t);
    if (rc) return rc;
    for (int k = 0; k < 5; ++k) c->last[k] = t[k];
    c->last_step = c->folded ? c->steps - 1 : c->steps;
    if (!isfinite(t[0]) || !isfinite(t[1]) || !isfinite(t[2]) || !isfinite(t[3])) {
        c->sticky = LBM_E_DIVERGED;
        return fail(c, LBM_E_DIVERGED, "non-finite mass or momentum (simulation diverged)");
    }
    if (t[4] > 0.0) {
        c->sticky = LBM_E_DOMAIN;
        return fail(c, LBM_E_DOMAIN, "density left the EOS domain (rho <= 0 or b*rho >= 1) at " +
                                         std::to_string((long long)t[4]) + " nodes");
    }
    return LBM_OK;
}

void fused_step(lbm_ctx *c) {
    for (const FusedSeg &sg : c->segs)
        sg.fn(c->stream, c->A, c->B, c->g, FusedMask{c->links, c->pflags, c->qlo}, params_ptr(c), sg.fg);
}

// the two-pass step, or the D2Q9 single pass, from lattice a into b on stream s
void unfused_step(lbm_ctx *c, hipStream_t s, const void *a, void *b) {
    if (c->single) {
        c->ks.single(s, a, b, c->g, c->mask, params_ptr(c));
    } else {
        c->ks.moments(s, a, c->g, c->mask, params_ptr(c), c->rho, c->gfl, c->partials);
        c->ks.collide(s, a, b, c->g, c->mask, params_ptr(c), c->rho, c->gfl);
    }
}

int one_step(lbm_ctx *c) {
    ++c->steps;
    if (c->fused) {
        fused_step(c);
        c->folded = c->fold;
    } else {
        unfused_step(c, c->stream, c->A, c->B);
    }
    void *t = c->A; c->A = c->B; c->B = t;
    return LBM_OK;
}

// Steps off the fused kernel (the D2Q9 single pass, the two-pass step) per captured graph.
// Even, so that a replay leaves the two lattices in the roles it found them in; 32 steps
// make the host's launch cost per step small next to a grid's own time down to a few
// thousand nodes.
constexpr int kGraphSteps = 32;

// Captures kGraphSteps steps from the current lattice on the context's own stream (never the
// caller's, which may itself be capturing). The graph holds kernels only.
int capture_steps(lbm_ctx *c) {
    HIP_OR_FAIL(c, hipStreamSynchronize(c->own));   // once per context: nothing queued under the capture
    HIP_OR_FAIL(c, hipStreamBeginCapture(c->own, hipStreamCaptureModeThreadLocal));
    void *a = c->A, *b = c->B;
    for (int s = 0; s < kGraphSteps; ++s) {
        unfused_step(c, c->own, a, b);
        std::swap(a, b);
    }
    const hipError_t le = hipGetLastError();
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(c->own, &graph);
    hipError_t ie = hipSuccess;
    if (le == hipSuccess && ee == hipSuccess) ie = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);   // the executable graph does not need it
    const hipError_t e = le != hipSuccess ? le : (ee != hipSuccess ? ee : ie);
    if (e != hipSuccess) {
        c->gexec = nullptr;
        return fail(c, LBM_E_HIP, std::string("capturing the step graph failed: ") + hipGetErrorString(e));
    }
    c->gA = c->A;
    return LBM_OK;
}

// n steps with no check among them. Steps off the fused kernel replay the captured block
// while at least kGraphSteps steps remain (after one plain step when the lattices are in the
// other roles), unless the context's stream is being captured by the caller; the rest go one
// by one.
int run_steps(lbm_ctx *c, int64_t n) {
    if (c->use_graph && n >= kGraphSteps) {
        hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
        HIP_OR_FAIL(c, hipStreamIsCapturing(c->stream, &st));
        if (st == hipStreamCaptureStatusNone) {
            if (!c->gexec) {
                const int rc = capture_steps(c);
                if (rc) return rc;
            }
            if (c->A != c->gA) {
                one_step(c);
                --n;
            }
            for (; n >= kGraphSteps; n -= kGraphSteps) {
                HIP_OR_FAIL(c, hipGraphLaunch(c->gexec, c->stream));
                c->steps += kGraphSteps;
            }
        }
    }
    for (; n > 0; --n) one_step(c);
    return LBM_OK;
}

// rows of `words` 4-byte words from pitch sp to pitch dp (both in words)
__global__ void k_repitch(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst, long long words, long long sp,
                          long long dp, long long rows) {
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= words * rows) return;
    const long long r = k / words, w = k - r * words;
    dst[r * dp + w] = src[r * sp + w];
}

// nodes of the user layout (x fastest, rows of nx)
size_t user_nodes(const lbm_ctx *c) { return (size_t)c->g.nx * c->g.ny * c->g.nz; }

// Copy between the user layout (rows of nx elements) and the device layout (rows of px):
// ny nz rows of nx elements of `elem` bytes, on the context stream.
hipError_t copy_rows(lbm_ctx *c, void *dst, const void *src, size_t elem, hipMemcpyKind kind) {
    const bool to_dev = kind == hipMemcpyHostToDevice;
    const size_t upitch = (size_t)c->g.nx * elem, dpitch = (size_t)c->g.px * elem;
    const size_t rows = (size_t)c->g.ny * c->g.nz, bytes = upitch * rows;
    if (upitch == dpitch)   // unpadded rows: one contiguous copy
        return hipMemcpyAsync(dst, src, bytes, kind, c->stream);
    // padded rows: repack on the device through a contiguous buffer and copy that in one
    // piece (a 2D copy to pageable host memory goes row by row, ~0.3 GB/s)
    hipError_t e;
    if (!c->pack && (e = hipMalloc(&c->pack, user_nodes(c) * sizeof(double))) != hipSuccess) {
        c->pack = nullptr;
        return e;
    }
    const long long words = (long long)(upitch / 4), up = words, dp = (long long)(dpitch / 4);
    const dim3 grid((unsigned)((words * (long long)rows + 255) / 256));
    if (to_dev) {
        if ((e = hipMemcpyAsync(c->pack, src, bytes, kind, c->stream)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_repitch, grid, dim3(256), 0, c->stream, (const uint32_t *)c->pack, (uint32_t *)dst, words,
                           up, dp, (long long)rows);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_repitch, grid, dim3(256), 0, c->stream, (const uint32_t *)src, (uint32_t *)c->pack, words, dp,
                       up, (long long)rows);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return hipMemcpyAsync(dst, c->pack, bytes, kind, c->stream);
}

int env_int(const char *name, int dflt) {
    const char *v = getenv(name);
    return (v && *v) ? atoi(v) : dflt;
}

}  // namespace

extern "C" {

int lbm_create(const lbm_params *p, lbm_ctx **out) {
    if (!out) return fail(nullptr, LBM_E_INVAL, "out is NULL");
    *out = nullptr;
    std::string why;
    if (!validate_params(p, &why)) return fail(nullptr, LBM_E_INVAL, why);
    lbm_ctx *c = new (std::nothrow) lbm_ctx;
    if (!c) return fail(nullptr, LBM_E_NOMEM, "host allocation failed");
    c->p = *p;
    c->p.mask = nullptr;
    c->p.rho_wall_field = nullptr;
    c->p.link_q = nullptr;
    c->D = p->lattice == LBM_D3Q27 ? 3 : 2;
    c->Q = c->D == 3 ? 27 : 9;
    c->fp64 = p->precision == LBM_FP64;
    c->masked = p->mask != nullptr;
    c->sbytes = c->fp64 ? 8 : 4;
    {
        // rows padded to whole 128-byte lines (32 nodes) from nx = 64 on, so that a 64-node
        // row load touches two cache lines, not three; LBM2P_PITCH_ALL=1 pads any nx
        const int nx = p->nx, nz = c->D == 3 ? p->nz : 1;
        const int px = (nx >= 64 || env_int("LBM2P_PITCH_ALL", 0)) ? (nx + 31) / 32 * 32 : nx;
        if ((double)px * p->ny * nz >= 2147483647.0) {
            delete c;
            return fail(nullptr, LBM_E_INVAL, "grid larger than 2^31 nodes with its rows padded");
        }
        c->g = make_geom(nx, p->ny, nz, px);
    }
    fill_params(p, &c->pd);
    fill_params(p, &c->pf);
    c->ks = kernel_set(c->D, c->fp64, c->masked);
    c->nblk = moment_block_count(c->D, c->g);
    // single-pass z-march for D3Q27 (LBM2P_TWO_PASS=1 forces the two-pass step;
    // LBM2P_FUSED_TX / _TY / _TZ override the tile shape and z-chunk length). By default
    // the z-chunks are as long as possible while every CU still gets a work item: each
    // chunk re-reads a four-plane z halo and runs a five-plane prologue.
    const int tx = env_int("LBM2P_FUSED_TX", 64), ty = env_int("LBM2P_FUSED_TY", 8);
    int cus = 256;
    {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            cus = n;
    }
    const long long tiles = (long long)((c->g.nx + tx - 1) / tx) * ((c->g.ny + ty - 1) / ty);
    // Small grids: a work item marches its planes one after another, so when even 16-plane
    // z-chunks give fewer items than CUs, the two-pass step, parallel over all nodes, is
    // faster (per step, FP32 at 32^3, 64^3, 96^3: 94, 90, 104 us single-pass against 17, 25,
    // 84 two-pass; FP64 162, 178, 211 against 22, 50, 200; at 128^3 the single pass wins, 129
    // against 162 FP32). LBM2P_FUSED=1 takes the single-pass step at any size.
    const bool few_items = tiles * std::max(1, c->g.nz / 16) < cus;
    if (c->D == 3 && !env_int("LBM2P_TWO_PASS", 0) && (!few_items || env_int("LBM2P_FUSED", 0))) {
        // Chunk length for a run of len planes. Each work item (tile x chunk) marches its
        // planes after a five-plane prologue; items run in rounds of one per CU. The number
        // of chunks minimises rounds x (planes per chunk + 6), chunks of >= 16 planes: long
        // chunks, but no last round that leaves most CUs idle (288 tiles on 256 CUs in one
        // chunk would take two full rounds' time for 1.1 rounds' work). Chunks stay within
        // 320 planes: over longer marches neighbouring tiles drift apart in z and the halo
        // lines they share leave L2 between the two reads (600^3: 600-plane chunks 14.7,
        // 300-plane chunks 15.2 GLUPS).
        auto chunk = [&](int len) {
            long long best = 1, cost = -1;
            for (long long nzc = std::max(1, (len + 319) / 320); nzc <= std::max(1, len / 16); ++nzc) {
                const long long rounds = (tiles * nzc + cus - 1) / cus;
                const long long c = rounds * ((len + nzc - 1) / nzc + 6);
                if (cost < 0 || c < cost) { cost = c; best = nzc; }
            }
            const int tz = env_int("LBM2P_FUSED_TZ", (int)((len + best - 1) / best));
            return tz > 0 ? tz : 32;
        };
        // the fused kernel addresses a lattice through one buffer resource, through two
        // (FP64, populations 0-13 and 14-26) when it exceeds the 4 GiB reach of one, and
        // beyond that through one resource per group of four (FP32) or two (FP64)
        // populations (LBM2P_FUSED_GROUPED=1 forces the last)
        const unsigned long long pop = (unsigned long long)c->g.qs * c->sbytes;
        int lat = 27 * pop < 0xFFFFFFFFull ? 0 : (c->fp64 && 14 * pop < 0xFFFFFFFFull ? 1 : 2);
        if (env_int("LBM2P_FUSED_GROUPED", 0)) lat = 2;
        if (lat == 2 && (c->fp64 ? 2 : 4) * pop >= 0xFFFFFFFFull) lat = -1;   // no fused step this large
        if (lat >= 0) {
            const FusedLaunch plain = fused_launcher(c->fp64, false, tx, ty, lat, false);
            const FusedLaunch walls = c->masked ? fused_launcher(c->fp64, true, tx, ty, lat, p->link_q != nullptr)
                                                : nullptr;
            const int nz = c->g.nz;
            if (!c->masked) {
                if (plain) c->segs.push_back({plain, fused_grid(c->g, tx, ty, chunk(nz), 0, nz)});
            } else if (walls) {
                // A plane is collided, staged and pulled from within three planes of itself,
                // so planes with no solid node in z-3..z+3 run the unmasked kernel; maximal
                // runs of equal kind become the launches of a step
                const size_t nxy = (size_t)c->g.nx * c->g.ny;
                std::vector<char> has(nz, 0), near(nz, 0);
                for (int z = 0; z < nz; ++z)
                    for (size_t q = 0; q < nxy && !has[z]; ++q) has[z] = p->mask[(size_t)z * nxy + q] ? 1 : 0;
                for (int z = 0; z < nz; ++z)
                    for (int d = -3; d <= 3 && !near[z]; ++d) near[z] = has[((z + d) % nz + nz) % nz];
                for (int zb = 0; zb < nz;) {
                    int ze = zb + 1;
                    while (ze < nz && near[ze] == near[zb]) ++ze;
                    const FusedLaunch fn = near[zb] || !plain ? walls : plain;
                    c->segs.push_back({fn, fused_grid(c->g, tx, ty, chunk(ze - zb), zb, ze)});
                    zb = ze;
                }
            }
            // one launch per round of work items (one item per CU); every item of a step owns
            // one row of the FP64 totals, numbered across the plane runs
            std::vector<FusedSeg> rounds;
            int slot0 = 0;
            for (const FusedSeg &sg : c->segs) {
                for (FusedGrid w : fused_windows(sg.fg, cus)) {
                    w.slot0 = slot0;
                    rounds.push_back({sg.fn, w});
                }
                slot0 += sg.fg.items;
            }
            c->segs = rounds;
            c->nfslots = slot0;
            if (!c->segs.empty()) c->fused = c->segs[0].fn;
        }
    }
    // D2Q9 steps in one pass (LBM2P_TWO_PASS=1: the moment pass, then the collide)
    c->single = c->D == 2 && !env_int("LBM2P_TWO_PASS", 0) && c->ks.single;
    // unfused steps replay captured blocks of steps (LBM2P_GRAPH=0: every step launched)
    c->use_graph = !c->fused && env_int("LBM2P_GRAPH", 1) != 0;
    const size_t N = (size_t)c->g.N;
    const size_t cbytes = c->fp64 ? 8 : 4;
    hipError_t e;
    if ((e = hipGetDevice(&c->device)) != hipSuccess || (e = hipStreamCreate(&c->own)) != hipSuccess) {
        free_ctx(c);
        return fail(nullptr, LBM_E_HIP, std::string("HIP initialisation failed: ") + hipGetErrorString(e));
    }
    c->stream = c->own;
    if ((e = device_scratch(c->device, &c->scratch)) != hipSuccess) {
        free_ctx(c);
        return fail(nullptr, LBM_E_HIP, std::string("address of the device scratch: ") + hipGetErrorString(e));
    }
    for (FusedSeg &sg : c->segs) sg.fg.partials = nullptr;   // set once fpart exists
    const size_t pop = (size_t)c->Q * (size_t)c->g.qs * c->sbytes;
    if (hipMalloc(&c->A, pop) != hipSuccess || hipMalloc(&c->B, pop) != hipSuccess ||
        hipMalloc(&c->rho, N * cbytes) != hipSuccess || hipMalloc(&c->gfl, (size_t)c->D * N * cbytes) != hipSuccess ||
        hipMalloc((void **)&c->partials, (size_t)c->nblk * kPartialSlots * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&c->rscratch, (size_t)std::max(reduce_scratch_rows(c->nblk), reduce_scratch_rows(c->nfslots)) *
                                             kPartialSlots * sizeof(double)) != hipSuccess ||
        (c->nfslots && hipMalloc((void **)&c->fpart, (size_t)c->nfslots * kPartialSlots * sizeof(double)) != hipSuccess) ||
        hipMalloc((void **)&c->io, (size_t)(1 + c->D) * N * sizeof(double)) != hipSuccess) {
        free_ctx(c);
        return fail(nullptr, LBM_E_NOMEM, "device allocation failed (" + std::to_string(2 * pop >> 20) + " MiB of populations)");
    }
    if (hipHostMalloc((void **)&c->htot, 8 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer((void **)&c->htot_dev, c->htot, 0) != hipSuccess) {
        free_ctx(c);
        return fail(nullptr, LBM_E_NOMEM, "pinned host allocation of the watchdog totals failed");
    }
    // the FP32 single-pass kernels without mask accumulate the totals of their input state
    c->fold = c->fused && !c->masked && !c->fp64 && c->nfslots > 0;
    for (FusedSeg &sg : c->segs) sg.fg.partials = c->fold ? c->fpart : nullptr;
    if (p->rho_wall_field) {   // per-node wall densities (solid entries are the ones used)
        c->wall = c->fp64 ? (void *)upload_wall_field<double>(p->rho_wall_field, c->g)
                          : (void *)upload_wall_field<float>(p->rho_wall_field, c->g);
        if (!c->wall) {
            free_ctx(c);
            return fail(nullptr, LBM_E_NOMEM, "device allocation of the wall density field failed");
        }
        if (c->fp64) c->pd.rho_wf = (const double *)c->wall;
        else c->pf.rho_wf = (const float *)c->wall;
    }
    if (p->link_q) {   // wall fractions of the links into solid nodes
        c->lq = c->fp64 ? (void *)upload_link_q<double>(p->link_q, c->Q, c->g)
                        : (void *)upload_link_q<float>(p->link_q, c->Q, c->g);
        if (!c->lq) {
            free_ctx(c);
            return fail(nullptr, LBM_E_NOMEM, "device allocation of the link fractions failed");
        }
        if (c->fp64) c->pd.link_q = (const double *)c->lq;
        else c->pf.link_q = (const float *)c->lq;
    }
    if (c->masked) {
        if (hipMalloc((void **)&c->mask, N) != hipSuccess) {
            free_ctx(c);
            return fail(nullptr, LBM_E_NOMEM, "device allocation of the mask failed");
        }
        const std::vector<uint8_t> mp = pitched<uint8_t>(p->mask, c->g);
        if ((e = hipMemcpy(c->mask, mp.data(), N, hipMemcpyHostToDevice)) != hipSuccess) {
            free_ctx(c);
            return fail(nullptr, LBM_E_HIP, std::string("mask upload failed: ") + hipGetErrorString(e));
        }
        if (c->fused) {   // solid-neighbour bits: one word per node instead of 27 mask reads per pull
            if (hipMalloc((void **)&c->links, N * sizeof(uint32_t)) != hipSuccess) {
                free_ctx(c);
                return fail(nullptr, LBM_E_NOMEM, "device allocation of the link mask failed");
            }
            fused_links(c->stream, c->mask, c->links, c->g);
            if (c->lq) {   // which partner each interpolated wall link reads
                if (hipMalloc((void **)&c->qlo, N * sizeof(uint32_t)) != hipSuccess) {
                    free_ctx(c);
                    return fail(nullptr, LBM_E_NOMEM, "device allocation of the wall-link bits failed");
                }
                fused_qlo(c->stream, c->links, c->lq, c->fp64, c->qlo, c->g);
            }
            const int nz = c->g.nz, nxy = c->g.nx * c->g.ny;
            std::vector<uint32_t> has(nz, 0u), pf(nz, 0u);
            for (int z = 0; z < nz; ++z)
                for (int q = 0; q < nxy && !has[z]; ++q) has[z] = p->mask[(size_t)z * nxy + q] ? 1u : 0u;
            for (int z = 0; z < nz; ++z)
                pf[z] = has[z] | ((has[(z + nz - 1) % nz] | has[z] | has[(z + 1) % nz]) << 1);
            if (hipMalloc((void **)&c->pflags, nz * sizeof(uint32_t)) != hipSuccess) {
                free_ctx(c);
                return fail(nullptr, LBM_E_NOMEM, "device allocation of the plane flags failed");
            }
            if ((e = hipMemcpy(c->pflags, pf.data(), nz * sizeof(uint32_t), hipMemcpyHostToDevice)) != hipSuccess) {
                free_ctx(c);
                return fail(nullptr, LBM_E_HIP, std::string("plane flag upload failed: ") + hipGetErrorString(e));
            }
            if ((e = hipStreamSynchronize(c->stream)) != hipSuccess || (e = hipGetLastError()) != hipSuccess) {
                free_ctx(c);
                return fail(nullptr, LBM_E_HIP, std::string("link mask failed: ") + hipGetErrorString(e));
            }
        }
    }
    *out = c;
    return LBM_OK;
}

int lbm_init_fields(lbm_ctx *c, const double *rho, const double *u) {
    if (!c || !rho) return fail(c, LBM_E_INVAL, "context or rho is NULL");
    const size_t N = (size_t)c->g.N, Nu = user_nodes(c);
    for (size_t n = 0; n < Nu; ++n) {
        if (!(rho[n] > 0.0) || !isfinite(rho[n])) return fail(c, LBM_E_DOMAIN, "initial density must be finite and > 0");
    }
    HIP_OR_FAIL(c, copy_rows(c, c->io, rho, sizeof(double), hipMemcpyHostToDevice));
    if (u)
        for (int a = 0; a < c->D; ++a)
            HIP_OR_FAIL(c, copy_rows(c, c->io + N + (size_t)a * N, u + (size_t)a * Nu, sizeof(double),
                                     hipMemcpyHostToDevice));
    const long long count = (long long)c->Q * c->g.qs;
    c->ks.fill_zero(c->stream, c->A, count);
    c->ks.fill_zero(c->stream, c->B, count);
    c->ks.init(c->stream, c->A, c->g, c->mask, params_ptr(c), c->rho, c->io, u ? c->io + N : nullptr);
    HIP_OR_FAIL(c, hipGetLastError());
    c->sticky = 0;
    c->initialized = true;
    c->folded = false;
    c->steps = 0;
    double t[5];
    int rc = reduce_state(c, t);
    if (rc) return rc;
    c->M0 = t[0];
    return watchdog(c);
}

int lbm_step(lbm_ctx *c, int64_t n) {
    if (!c) return fail(c, LBM_E_INVAL, "context is NULL");
    if (n < 0) return fail(c, LBM_E_INVAL, "negative step count");
    if (!c->initialized) return fail(c, LBM_E_STATE, "lbm_step before lbm_init_fields");
    if (c->sticky) return c->sticky;
    const int ce = c->p.check_every;
    // runs between watchdog checks: after every ce steps of this call, and at its end
    for (int64_t done = 0; done < n;) {
        const int64_t run = ce > 0 ? std::min<int64_t>(n - done, ce - done % ce) : n - done;
        int rc = run_steps(c, run);
        if (rc) return rc;
        done += run;
        if (ce > 0 && done % ce == 0 && done < n && (rc = watchdog(c))) return rc;
    }
    HIP_OR_FAIL(c, hipGetLastError());
    if (ce >= 0) return watchdog(c);
    return LBM_OK;
}

int lbm_step_timed(lbm_ctx *c, int64_t n, double ms[3], int64_t launches[2]) {
    if (!c || !ms || !launches) return fail(c, LBM_E_INVAL, "NULL argument");
    if (!c->initialized) return fail(c, LBM_E_STATE, "lbm_step_timed before lbm_init_fields");
    if (c->sticky) return c->sticky;
    hipEvent_t ev[3];
    for (auto &e : ev) HIP_OR_FAIL(c, hipEventCreate(&e));
    hipEvent_t tot0, tot1;
    HIP_OR_FAIL(c, hipEventCreate(&tot0));
    HIP_OR_FAIL(c, hipEventCreate(&tot1));
    double acc[2] = {0.0, 0.0};
    HIP_OR_FAIL(c, hipEventRecord(tot0, c->stream));
    for (int64_t t = 0; t < n; ++t) {
        HIP_OR_FAIL(c, hipEventRecord(ev[0], c->stream));
        if (!c->fused && !c->single)
            c->ks.moments(c->stream, c->A, c->g, c->mask, params_ptr(c), c->rho, c->gfl, c->partials);
        HIP_OR_FAIL(c, hipEventRecord(ev[1], c->stream));
        if (c->fused) {
            fused_step(c);
            c->folded = c->fold;
        } else if (c->single) {
            c->ks.single(c->stream, c->A, c->B, c->g, c->mask, params_ptr(c));
        } else {
            c->ks.collide(c->stream, c->A, c->B, c->g, c->mask, params_ptr(c), c->rho, c->gfl);
        }
        ++c->steps;
        HIP_OR_FAIL(c, hipEventRecord(ev[2], c->stream));
        HIP_OR_FAIL(c, hipEventSynchronize(ev[2]));
        float a = 0.f, b = 0.f;
        HIP_OR_FAIL(c, hipEventElapsedTime(&a, ev[0], ev[1]));
        HIP_OR_FAIL(c, hipEventElapsedTime(&b, ev[1], ev[2]));
        acc[0] += a;
        acc[1] += b;
        void *tmp = c->A; c->A = c->B; c->B = tmp;
    }
    HIP_OR_FAIL(c, hipEventRecord(tot1, c->stream));
    HIP_OR_FAIL(c, hipEventSynchronize(tot1));
    float tt = 0.f;
    HIP_OR_FAIL(c, hipEventElapsedTime(&tt, tot0, tot1));
    for (auto &e : ev) (void)hipEventDestroy(e);
    (void)hipEventDestroy(tot0);
    (void)hipEventDestroy(tot1);
    ms[0] = acc[0];
    ms[1] = acc[1];
    ms[2] = tt;
    launches[0] = c->fused || c->single ? 0 : n;
    launches[1] = n;
    return LBM_OK;
}

int lbm_moments(lbm_ctx *c, double *rho, double *U, double totals[4]) {
    if (!c) return fail(c, LBM_E_INVAL, "context is NULL");
    if (!c->initialized) return fail(c, LBM_E_STATE, "lbm_moments before lbm_init_fields");
    double t[5];
    int rc = reduce_state(c, t);    // also refreshes rho and g of the current state
    if (rc) return rc;
    if (totals) for (int k = 0; k < 4; ++k) totals[k] = t[k];
    if (rho || U) {
        const size_t N = (size_t)c->g.N;
        c->ks.output(c->stream, c->A, c->g, c->mask, params_ptr(c), c->rho, c->gfl, c->io, c->io + N);
        HIP_OR_FAIL(c, hipGetLastError());
        const size_t Nu = user_nodes(c);
        if (rho) HIP_OR_FAIL(c, copy_rows(c, rho, c->io, sizeof(double), hipMemcpyDeviceToHost));
        if (U)
            for (int a = 0; a < c->D; ++a)
                HIP_OR_FAIL(c, copy_rows(c, U + (size_t)a * Nu, c->io + N + (size_t)a * N, sizeof(double),
                                         hipMemcpyDeviceToHost));
        HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    }
    return LBM_OK;
}

int lbm_moments_noalloc(lbm_ctx *c, double *rho, double *U, double *totals) {
    if (!c) return fail(c, LBM_E_INVAL, "context is NULL");
    // the moment pass writes one partial row per workgroup; the tree's levels follow them
    const size_t rows = (size_t)c->nblk + (size_t)reduce_scratch_rows(c->nblk);
    const size_t need = rows * kPartialSlots * sizeof(double);
    if (need > kScratchBytes)
        return fail(c, LBM_E_INVAL, "lbm_moments_noalloc: the grid needs " + std::to_string(need) +
                                        " bytes of scratch, more than its " + std::to_string(kScratchBytes) +
                                        " (use lbm_moments)");
    if (!c->initialized) return fail(c, LBM_E_STATE, "lbm_moments_noalloc before lbm_init_fields");
    double *part = c->scratch, *tree = c->scratch + (size_t)c->nblk * kPartialSlots;
    c->ks.moments(c->stream, c->A, c->g, c->mask, params_ptr(c), c->rho, c->gfl, part);
    if (totals) launch_reduce(c->stream, part, c->nblk, tree, totals);
    if (rho || U) {
        // unpadded rows: the output pass writes the caller's buffers (the context's staging
        // takes a field the caller did not ask for); padded rows: staging, then a repack
        const size_t N = (size_t)c->g.N;
        const bool padded = c->g.px != c->g.nx;
        c->ks.output(c->stream, c->A, c->g, c->mask, params_ptr(c), c->rho, c->gfl,
                     (padded || !rho) ? c->io : rho, (padded || !U) ? c->io + N : U);
        if (padded) {
            const long long words = 2LL * c->g.nx, sp = 2LL * c->g.px, yz = (long long)c->g.ny * c->g.nz;
            auto repack = [&](const double *src, double *dst, long long rows_) {
                const dim3 grid((unsigned)((words * rows_ + 255) / 256));
                hipLaunchKernelGGL(k_repitch, grid, dim3(256), 0, c->stream, (const uint32_t *)src, (uint32_t *)dst,
                                   words, sp, words, rows_);
            };
            if (rho) repack(c->io, rho, yz);
            if (U) repack(c->io + N, U, c->D * yz);   // the D components are consecutive in both layouts
        }
    }
    HIP_OR_FAIL(c, hipGetLastError());
    return LBM_OK;
}

int lbm_pressure_tensor(lbm_ctx *c, double *P) {
    if (!c || !P) return fail(c, LBM_E_INVAL, "NULL argument");
    if (!c->initialized) return fail(c, LBM_E_STATE, "lbm_pressure_tensor before lbm_init_fields");
    const int nc = c->D * (c->D + 1) / 2;
    const size_t N = (size_t)c->g.N, Nu = user_nodes(c);
    if (!c->ptens && hipMalloc((void **)&c->ptens, (size_t)nc * N * sizeof(double)) != hipSuccess) {
        c->ptens = nullptr;
        return fail(c, LBM_E_NOMEM, "device allocation of the pressure tensor failed");
    }
    double t[5];
    int rc = reduce_state(c, t);    // rho of the current state
    if (rc) return rc;
    c->ks.pressure(c->stream, c->A, c->g, c->mask, params_ptr(c), c->rho, c->ptens);
    HIP_OR_FAIL(c, hipGetLastError());
    for (int k = 0; k < nc; ++k)
        HIP_OR_FAIL(c, copy_rows(c, P + (size_t)k * Nu, c->ptens + (size_t)k * N, sizeof(double), hipMemcpyDeviceToHost));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

void lbm_destroy(lbm_ctx *c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_ctx(c);
}

const char *lbm_last_error(const lbm_ctx *c) { return c ? c->err.c_str() : g_create_err.c_str(); }

int lbm_last_check(const lbm_ctx *c, double out[5], int64_t *state_step) {
    if (!c || !out) return LBM_E_INVAL;
    if (c->last_step < 0) return LBM_E_STATE;
    for (int k = 0; k < 5; ++k) out[k] = c->last[k];
    if (state_step) *state_step = c->last_step;
    return LBM_OK;
}

int lbm_set_stream(lbm_ctx *c, void *hip_stream) {
    if (!c) return fail(c, LBM_E_INVAL, "context is NULL");
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    c->stream = hip_stream ? (hipStream_t)hip_stream : c->own;
    return LBM_OK;
}

int64_t lbm_population_bytes(const lbm_ctx *c) {
    return c ? (int64_t)c->Q * (int64_t)user_nodes(c) * (int64_t)c->sbytes : 0;
}

int lbm_get_populations(lbm_ctx *c, void *host) {
    if (!c || !host) return fail(c, LBM_E_INVAL, "NULL argument");
    if (!c->initialized) return fail(c, LBM_E_STATE, "no state to checkpoint");
    const size_t row = user_nodes(c) * c->sbytes;
    for (int i = 0; i < c->Q; ++i)
        HIP_OR_FAIL(c, copy_rows(c, (char *)host + i * row, (char *)c->A + (size_t)i * c->g.qs * c->sbytes, c->sbytes,
                                 hipMemcpyDeviceToHost));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int lbm_set_populations(lbm_ctx *c, const void *host) {
    if (!c || !host) return fail(c, LBM_E_INVAL, "NULL argument");
    const size_t row = user_nodes(c) * c->sbytes;
    for (int i = 0; i < c->Q; ++i)
        HIP_OR_FAIL(c, copy_rows(c, (char *)c->A + (size_t)i * c->g.qs * c->sbytes, (const char *)host + i * row,
                                 c->sbytes, hipMemcpyHostToDevice));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    c->initialized = true;
    c->sticky = 0;
    c->folded = false;
    c->steps = 0;
    return watchdog(c);
}

int lbm_velocities(int lattice, int *c) {
    if (!c || (lattice != LBM_D2Q9 && lattice != LBM_D3Q27)) return fail(nullptr, LBM_E_INVAL, "bad argument");
    const int D = lattice == LBM_D3Q27 ? 3 : 2, Q = D == 3 ? 27 : 9;
    for (int i = 0; i < Q; ++i)
        for (int a = 0; a < 3; ++a) c[3 * i + a] = D == 3 ? Lat<3>::c(i, a) : Lat<2>::c(i, a);
    return Q;
}

int lbm_coexistence(const lbm_params *p, double out[4]) {
    if (!p || !out) return fail(nullptr, LBM_E_INVAL, "NULL argument");
    HostEos e(p->eos, p->a, p->b, p->R, p->acentric, p->T_reduced);
    double rv, rl, ps;
    if (coexistence(e, &rv, &rl, &ps)) return fail(nullptr, LBM_E_DOMAIN, "no van der Waals loop at this temperature");
    out[0] = rv; out[1] = rl; out[2] = ps;
    out[3] = (p->eos == LBM_EOS_SC1 || p->eos == LBM_EOS_SC2) ? e.aa : e.T;   // Shan-Chen: the coupling G
    return LBM_OK;
}

int lbm_surface_tension(const lbm_params *p, double *sigma) {
    if (!p || !sigma || !(p->kappa >= 0)) return fail(nullptr, LBM_E_INVAL, "bad argument");
    HostEos e(p->eos, p->a, p->b, p->R, p->acentric, p->T_reduced);
    if (surface_tension(e, p->kappa, sigma)) return fail(nullptr, LBM_E_DOMAIN, "no van der Waals loop at this temperature");
    return LBM_OK;
}

int lbm_eos_pressure(const lbm_params *p, const double *rho, int64_t n, double *P) {
    if (!p || (n > 0 && (!rho || !P)) || n < 0) return fail(nullptr, LBM_E_INVAL, "bad argument");
    HostEos e(p->eos, p->a, p->b, p->R, p->acentric, p->T_reduced);
    for (int64_t k = 0; k < n; ++k) P[k] = e.P(rho[k]);
    return LBM_OK;
}

int lbm_kappa_for_width(const lbm_params *p, double width, double *kappa) {
    if (!p || !kappa || !(width > 0)) return fail(nullptr, LBM_E_INVAL, "bad argument");
    HostEos e(p->eos, p->a, p->b, p->R, p->acentric, p->T_reduced);
    if (kappa_for_width(e, width, kappa)) return fail(nullptr, LBM_E_DOMAIN, "no van der Waals loop at this temperature");
    return LBM_OK;
}

}  // extern "C"
