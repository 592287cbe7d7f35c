// Launch arguments of the path kernels, shared by the single-view entry
// points and the multi-view batches.
#pragma once
#include <cstdint>

#include "dr_common.h"

namespace dr {

constexpr int BS = 64;   // one wave per block

struct RenderArgs {
    int spp, depth, M, Ww;
    int debug_unit;    // unit whose secondary samples are printed (-1: none)
    unsigned long long* counters;   // [5] work counters, or null
    uint32_t k0, k1, view, terms;
    const uint8_t* mask;
    int* ck_tri;       // [3][M] triangle at path vertices 0, 1, 2 (-1: none)
    float* ck_x;       // [3][M][3] their positions
    uint8_t* ck_vis;   // [M]
    // gradient shards: block b adds into copy (b & (gshards - 1)) of the
    // gradient arrays (gstride floats apart) and of the camera accumulator
    // (12 floats apart); the copies are summed after the kernels
    int gshards;
    long gstride;
    int aov;           // 0: radiance; 1..7: geometry-buffer channel (the _aov kernels)
    int edge_t;        // point on a secondary edge: 0 uniform in t, 1 by the clamped cosine
    int cands;         // secondary edge selection: <= 1 one descent, M > 1 M-sample descent + reservoir
    float nee, nee_w;  // next event estimation for edges: probability of the strip strategy (0: off), strip width
};

// Learned-proposal mixture and harvest (the <.., MIX = true> kernel variants).
struct MixArgs {
    const float* q;          // [E] proposal distribution over edges
    const double* mcdf;      // [E + 1] mixture CDF of primary edges (total weight at [E])
    const double* qcdf;      // [E + 1] CDF of q
    const double* plen;      // [E] clipped screen length of primary edges
    float mix;               // weight of q
    int prim, sec;           // mixture on for primary / secondary edges
    float* estats;           // [E] harvest accumulator, or null
};

// Side-path query of the split backward: a secondary edge sample whose two
// one-sided radiances are traced by a dense kernel of their own.
struct SideQuery {
    float p[3], wp[3], wm[3];    // shading point, directions just off the edge on both sides
    uint32_t sid;                // pixel-sample id (Philox counter word)
    int edge;
    float pdf;                   // probability of the edge
    int k;                       // path vertex (0 = first hit)
    float te, pdf_t;             // edge parameter of the point and its density
};

struct SplitArgs {
    SideQuery* q;                // [cap]
    float2* res;                 // [cap] (radiance on the + side, on the - side)
    int* qidx;                   // [MAXD][M] query of (vertex, unit), -1 if none
    int* count;                  // [MAXD] queries appended per path vertex (segment kk starts at kk * M)
    int* vtri;                   // [MAXD - 2][M] triangle hit by traced path vertex kk + 1 >= 3, slot kk - 1 (-1: miss)
    float* vx;                   // [MAXD - 2][M][3] its position
};

// Everything one view of a batch needs on the device (fixed when the batch
// is created; buffers belong to the batch or, for images, to the caller).
struct BatchView {
    Cam k;
    RenderArgs a;
    TreeView tv;
    const PEdge* pe;         // [E] primary edge table
    const double* pcdf;      // [E + 1] its CDF (total at [E])
    float* image;            // [H][W] of the window
    const float* d_image;    // [H][W]
    float* camacc;           // [12]
    int reduce;              // spp divides 64: in-wave image reduction
};

// Work list of a batched launch: blocks of 64 units, view after view.
struct BatchLaunch {
    const BatchView* views;
    const int* boff;         // [n + 1] first block of each view
    int nviews, total;       // total blocks
    int chunk;               // blocks per work item
    int* queue;              // work-item counter of a persistent launch, or null
    int gshards;             // gradient copies (power of two): block b adds into copy b & (gshards - 1),
    long gstride;            // gstride floats apart; each view's camera accumulator has gshards x 12 floats
};

}  // namespace dr
