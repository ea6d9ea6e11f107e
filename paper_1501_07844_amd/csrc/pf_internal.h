// Internal interface between the C-ABI host code (pf_api.cpp) and the gfx950
// kernels (pf_kernels.hip).  Not installed; the public ABI is pseudoflow.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "pseudoflow.h"

namespace pf {

// Label-graph coupling in path-weight form.  Node A (0-based over the
// non-source nodes) and end-label L are linked by W[A][L], the sum over the
// paths A -> L of the products of edge weights (W = 1 on the diagonal of a
// leaf).  With it the top-down flow excess is d_L = D_L + sum_A W[A][L] div q_A
// and the bottom-up implicit label is U_A = sum_L W[A][L] u_L.
struct GraphW {
    int32_t nl, nn;
    float w[PF_MAX_NODES][PF_MAX_LEAVES];
};

// Per-solve constants copied into the workspace before the first launch:
// the node capacities of PF_S_NODE_SCALAR and the path weights.
struct ConstBlock {
    float s_node[PF_MAX_NODES];
    float w[PF_MAX_NODES * PF_MAX_LEAVES];
};
constexpr int kConstFloats = PF_MAX_NODES + PF_MAX_NODES * PF_MAX_LEAVES;

// Arguments common to every per-iteration kernel.
struct StepArgs {
    int32_t nx, ny, nz;      // grid extents (nz == 1 in 2-D)
    int32_t V;               // voxels per problem
    int32_t B;               // problems
    int32_t nl, nn;          // end-labels, flows
    float inv_c;             // 1/c
    float ctau;              // c * tau
    int32_t s_mode;          // pf_s_mode (input check only)
    const float *D;          // [B][nl][V]
    const float *S;          // user field (shared or per node) or null
    // Capacity S_A at voxel v of problem b is Sp[b*s_sb + A*s_sa + v*s_sv]
    // for every s_mode (a single branch-free form): node constants come from
    // the workspace copy with strides (0, 1, 0), a shared field has
    // (V, 0, 1) and a per-node field (nn*V, V, 1).
    const float *Sp;
    int64_t s_sb, s_sa, s_sv;
    const float *W;          // workspace copy of ConstBlock::w, [A * PF_MAX_LEAVES + L]
    const void *ell_in;      // storage [B][nl][V]
    const void *q_in;        // storage [B][nn][nd][V]
    void *ell_out;           // == ell_in for in-place passes
    void *q_out;
};

// Workspace partition (byte offsets from the workspace base).
struct Layout {
    size_t results;          // 8 doubles: E, P, simplex err, flow excess, ...
    size_t flags;            // 64 int32
    size_t consts;           // ConstBlock
    size_t partials;         // kPartials x 4 doubles
    size_t ell[2];           // label state, ping and pong
    size_t q[2];             // flow state, ping and pong
    size_t total;
};

// Buffers of one reverse step (float32).  The two-kernel reverse step
// updates lbar and pbar in place (in == out); the fused one reads the *_in
// and writes the *_out buffers (ping-pong), since its halo points read
// values that neighbouring blocks overwrite.
struct AdjArgs {
    const float *q_k;        // flows entering step k [B][nn][nd][V]
    const float *ell_next;   // log-labels after step k [B][nl][V]
    const float *lbar_in;    // [B][nl][V]
    float *lbar_out;
    const float *pbar_in;    // [B][nn][nd][V]
    float *pbar_out;
    float *sbar;             // accumulated capacity gradient: [B][V] (sum over
                             // the flows) when sbar_shared, else [B][nn][V]
    float *dbar;             // [B][nl][V], accumulated (the caller's dD)
    int32_t sbar_shared;
    int32_t first;           // last forward step: no later flow gradient
};

// Launch geometry of the fused kernel: (x, y) tiles times z chunks times problems.
struct FusedGeom {
    int32_t tiles_x, tiles_y, n_chunks, cz;
    long blocks;
};

constexpr int kPartials = 1024;
constexpr int kBlock = 256;

size_t storage_bytes(int storage);
// Storage elements per voxel for a group of n state fields: n for fp32,
// n rounded up to even for the 16-bit types (packed in pairs).
inline size_t state_fields(int n, int storage) {
    return storage == PF_FP32 ? (size_t)n : 2 * (size_t)((n + 1) / 2);
}
Layout make_layout(const pf_grid &g, int nl, int nn, int storage, bool pingpong);

// Launchers; return hipSuccess or the launch error.
hipError_t launch_upload(const ConstBlock &c, float *dst, hipStream_t s);
hipError_t launch_init(const StepArgs &a, int nd, int storage, float ell0, hipStream_t s);
hipError_t launch_label(const StepArgs &a, bool ident, int nd, int storage, hipStream_t s);
hipError_t launch_flow(const StepArgs &a, bool ident, int nd, int storage, hipStream_t s);
// whole 2-D problems in LDS: `iters` iterations per launch, one block per
// problem, state in place
constexpr int kLdsThreads = 1024;
constexpr int kLdsVox = 4;              // voxels per thread (V <= 4096)
constexpr int kLdsFloats = 40 * 1024;   // 160 KB of LDS per block
bool lds_supported(int nd, int nl, int nn, long V);
bool lds_preferred(int nd, int nl, int nn, long V, int batch);
hipError_t launch_lds(const StepArgs &a, bool ident, int storage, int iters, hipStream_t s);
// 2-D tiles with ghost zones in LDS: up to TileGeom::k iterations per launch,
// one block per owned tile and problem, ping-pong state
struct TileGeom {
    int32_t ox, oy;          // owned tile
    int32_t k;               // ghost zone width = iterations per launch at most
    int32_t rw, rh;          // region extents (owned + ghosts, clipped to the image)
    int32_t tiles_x, tiles_y;
};
// one voxel of the region per thread: up to 32 x 32, 24 x 24 for builds of
// more than 8 flows (their registers)
constexpr int tile_threads(int nn_build) { return nn_build > 8 ? 576 : 1024; }
bool tile_supported(int nd, int nl, int nn);
bool tile_preferred(int nd, int nl, int nn, long V, int batch);
TileGeom tile_geometry(int nx, int ny, int batch, int nn);
hipError_t launch_tile(const StepArgs &a, bool ident, int storage, int iters, hipStream_t s);
hipError_t launch_fused(const StepArgs &a, bool ident, int nd, int storage, hipStream_t s);
bool fused_supported(int nd, int nl, int nn, bool identity);
bool fused_preferred(int nd, int nl, int nn, bool identity, int storage);
FusedGeom fused_geometry(const StepArgs &a);
// two iterations per launch (3-D Potts, up to 8 labels), ping-pong state
hipError_t launch_fused2(const StepArgs &a, int storage, hipStream_t s);
bool fused2_supported(int nd, int nl, int nn, bool identity);
bool fused2_preferred(int nd, int nl, int nn, bool identity, int storage);
FusedGeom fused2_geometry(const StepArgs &a);
// one pass per iteration for 3-D label graphs: the flow step of iteration k,
// then the label step of iteration k + 1 (state between passes: labels one
// iteration ahead of the flows), ping-pong state
// `tail`: the last nl of the nn nodes are the end-labels in order, so their
// path-weight rows are unit vectors (the pass then skips their products)
hipError_t launch_flow_label(const StepArgs &a, int storage, bool tail, hipStream_t s);
bool flow_label_supported(int nd, int nl, int nn, bool identity);
bool flow_label_tail_supported(int nl, int nn, int storage);
bool flow_label_preferred(int nd, int nl, int nn, bool identity, int storage, bool tail);
// PF_KERNEL_AUTO's choice of a one-pass-per-iteration kernel (either kind);
// `tail` as for launch_flow_label (assumed by the queries that have no graph)
inline bool any_fused_preferred(int nd, int nl, int nn, bool identity, int storage, bool tail) {
    return fused_preferred(nd, nl, nn, identity, storage) ||
           flow_label_preferred(nd, nl, nn, identity, storage, tail);
}
FusedGeom flow_label_geometry(const StepArgs &a);
// tiles of width x rows voxels, z chunks, problems (the z-marching kernels);
// about `target` blocks, chunks of at least 16 planes
FusedGeom tile_geometry(const StepArgs &a, int width, int rows, long target = 512);
hipError_t launch_copy_state(const StepArgs &a, int nd, int storage, hipStream_t s);
hipError_t launch_energy(const StepArgs &a, bool ident, int nd, int storage,
                         double *partials, double *results, hipStream_t s);
hipError_t launch_export(const StepArgs &a, int nd, int storage, float *u, int32_t *labels,
                         float *q, hipStream_t s);
hipError_t launch_check(const StepArgs &a, int32_t *flag, hipStream_t s);
hipError_t launch_export_ell(const StepArgs &a, int storage, float *ell, hipStream_t s);
hipError_t launch_adj_flow(const StepArgs &a, const AdjArgs &g, bool ident, int nd, hipStream_t s);
hipError_t launch_adj_label(const StepArgs &a, const AdjArgs &g, bool ident, int nd, hipStream_t s);
hipError_t launch_adj_fused(const StepArgs &a, const AdjArgs &g, bool ident, int nd, hipStream_t s);
bool adj_fused_supported(int nd, int nl, int nn, bool identity);
bool adj_fused_preferred(int nd, int nx, int nl, int nn, bool identity);
hipError_t launch_fill(float *p, size_t n, float val, hipStream_t s);
hipError_t launch_copy_f(const float *a, float *b, size_t n, hipStream_t s);
// out[A] = sum over problems and voxels of sbar[B][nn][V] (fp64 accumulation)
hipError_t launch_sum_nodes(const float *sbar, int B, int nn, size_t V, float *out, hipStream_t s);

}  // namespace pf
