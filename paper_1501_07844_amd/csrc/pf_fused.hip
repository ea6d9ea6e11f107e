// Fused single-pass iteration for gfx950: one kernel per iteration reads the
// label and flow state once and writes the next state once (ping-pong
// buffers), instead of the label pass + flow pass that read the flows and
// labels twice.
//
// Dependencies of one iteration at voxel x (Algorithms 1 and 2):
//   label step at x needs the old flows at x and x - e_k (divergence);
//   flow step at x needs the NEW labels at x and x + e_k (forward gradient).
// A block therefore owns an FTX x FTY tile of (x, y) columns and marches a
// chunk of z planes.  Along z the forward neighbour is the thread's own next
// plane (kept in registers, together with the old q_z of the previous plane
// for the divergence).  Along x and y the new labels of the plane are
// exchanged through LDS; the labels one row past the tile (y) and one column
// past it (x) belong to the neighbouring tiles and are recomputed here by
// extra "halo" threads: one row of FTX threads for the row, and FTY threads
// of one more row for the column, so that no wavefront evaluates two points
// per plane.  A 128 x 4 tile (768 threads) reads fewer partially used cache
// lines for the halo column than 64 x 8 and measured 3% faster; both fit the
// register budget of three wavefronts per SIMD without spilling.  Each
// point's label step, flow step and rounding are the expressions of the
// two-pass kernels, so both variants give the same state bit for bit.
//
// Block -> tile mapping is XCD-aware: consecutive hardware block ids land on
// different XCDs, so they are remapped to give each XCD a contiguous range
// of tiles (neighbouring tiles then share that XCD's L2 for the halo reads).

#include <hip/hip_runtime.h>
#include <math.h>

#include "pf_device.h"
#include "pf_internal.h"

namespace pf {
namespace {

using namespace dev;

constexpr int FTX = 128;              // tile width (two wavefronts per row)
constexpr int FTY = 4;                // owned rows per tile
constexpr int FTHREADS = FTX * (FTY + 2);   // owned rows + the halo row + the halo column

// Label step at voxel (x, y, z) of problem b.  qzb holds the old q_z of every
// flow one plane below (ignored at z == 0).  Returns the new labels as the
// exponential of the stored-precision log-label (what the two-pass flow
// kernel reads back), the old flows at the voxel in qpt, and stores the new
// log-labels when `store`.  All loads are issued first, unconditionally.
template <int ND, int NLMAX, int NNMAX, bool IDENT, typename T>
__device__ __forceinline__ void label_point(const StepArgs &a, int b, int x, int y, int z,
                                            const float (&qzb)[NNMAX], bool store,
                                            float (&u)[NLMAX], float (&qpt)[NNMAX][ND]) {
    const size_t V = (size_t)a.V;
    const int v = (z * a.ny + y) * a.nx + x;
    const unsigned uv = (unsigned)v;
    const Coord c{x, y, z};
    int m[3];
    bool bwd[3];
    backward_offsets(c, a, m, bwd);
    const bool fwd[3] = {x < a.nx - 1, y < a.ny - 1, ND == 3 && z < a.nz - 1};
    float d[NLMAX], e[NLMAX], qm[NNMAX][3];
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        const int Lc = L < a.nl ? L : a.nl - 1;
        d[L] = ldf(field<float>(a.D, b, a.nl, Lc, V), uv);
        e[L] = ld_ell<T>(a.ell_in, b, a.nl, L, V, uv);
    }
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) {
        qpt[A][0] = ld_q<T, ND>(a.q_in, b, a.nn, A, 0, V, uv);
        qpt[A][1] = ld_q<T, ND>(a.q_in, b, a.nn, A, 1, V, uv);
        if constexpr (ND == 3) qpt[A][2] = ld_q<T, ND>(a.q_in, b, a.nn, A, 2, V, uv);
        qm[A][0] = ld_q<T, ND>(a.q_in, b, a.nn, A, 0, V, uv - (unsigned)m[0]);
        qm[A][1] = ld_q<T, ND>(a.q_in, b, a.nn, A, 1, V, uv - (unsigned)m[1]);
        qm[A][2] = ND == 3 ? qzb[A] : 0.f;
    }
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) {
        const float q0[3] = {qpt[A][0], qpt[A][1], ND == 3 ? qpt[A][ND - 1] : 0.f};
        add_excess<NLMAX, IDENT>(a, d, A, div_from<ND>(q0, qm[A], fwd, bwd));
    }
    entropic_step<NLMAX>(a, d, e);
    if (store) {
#pragma unroll
        for (int L = 0; L < NLMAX; L += 2) st_ell2<T>(a.ell_out, b, a.nl, L, V, uv, e[L], e[L + 1]);
    }
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) u[L] = __expf(roundtrip(e[L], static_cast<const T *>(nullptr)));
}

template <int ND, int NLMAX, int NNMAX, bool IDENT, typename T>
__global__ __launch_bounds__(FTHREADS) void k_fused(StepArgs a, FusedGeom g) {
    __shared__ float lds[NLMAX][FTY + 1][FTX + 1];
    const int row = threadIdx.x / FTX;   // tile row (FTY: halo row, FTY + 1: halo column)
    const int col = threadIdx.x % FTX;

    // XCD-aware block -> tile mapping
    const int nb = gridDim.x;
    const int pb = blockIdx.x;
    const int lb = (nb % 8 == 0) ? (pb % 8) * (nb / 8) + pb / 8 : pb;
    const int bx = lb % g.tiles_x;
    int r = lb / g.tiles_x;
    const int by = r % g.tiles_y;
    r /= g.tiles_y;
    const int ch = r % g.n_chunks;
    const int b = r / g.n_chunks;
    const int x0 = bx * FTX, y0 = by * FTY;
    const int zs = ch * g.cz;
    const int ze = min(a.nz, zs + g.cz);

    // point A: owned voxel column (rows 0 .. FTY-1), or the halo row past
    // the tile (row FTY); point B (row FTY+1): the column past the tile
    const int xa = x0 + col, ya = y0 + row;
    const bool va = row <= FTY && xa < a.nx && ya < a.ny;
    const bool own = row < FTY && va;
    const int xb = x0 + FTX, yb = y0 + col;
    const bool vb = row == FTY + 1 && col < FTY && xb < a.nx && yb < a.ny;

    const size_t V = (size_t)a.V;

    float ua[NLMAX], ub[NLMAX];
    float qa[NNMAX][ND], qb[NNMAX][ND];
    float qzb[NNMAX];
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) qzb[A] = 0.f;

    // prologue: labels of plane zs (point A and B), old q_z of plane zs - 1
    if (va) {
        if (ND == 3 && zs > 0) {
            const int vbelow = ((zs - 1) * a.ny + ya) * a.nx + xa;
#pragma unroll
            for (int A = 0; A < NNMAX; ++A)
                qzb[A] = ld_q<T, ND>(a.q_in, b, a.nn, A, ND - 1, V, (unsigned)vbelow);
        }
        label_point<ND, NLMAX, NNMAX, IDENT, T>(a, b, xa, ya, zs, qzb, own, ua, qa);
#pragma unroll
        for (int L = 0; L < NLMAX; ++L) lds[L][row][col] = ua[L];
    }
    if (vb) {
        if (ND == 3 && zs > 0) {
            const int vbelow = ((zs - 1) * a.ny + yb) * a.nx + xb;
#pragma unroll
            for (int A = 0; A < NNMAX; ++A)
                qzb[A] = ld_q<T, ND>(a.q_in, b, a.nn, A, ND - 1, V, (unsigned)vbelow);
        }
        label_point<ND, NLMAX, NNMAX, IDENT, T>(a, b, xb, yb, zs, qzb, false, ub, qb);
#pragma unroll
        for (int L = 0; L < NLMAX; ++L) lds[L][col][FTX] = ub[L];
    }
    __syncthreads();

    for (int z = zs; z < ze; ++z) {
        const bool has_next = z + 1 < a.nz;
        // capacities of the owned voxel, loaded ahead of the label step
        float sv[NNMAX];
        if (own) {
            const int v = (z * a.ny + ya) * a.nx + xa;
#pragma unroll
            for (int A = 0; A < NNMAX; ++A) sv[A] = smooth(a, b, A < a.nn ? A : a.nn - 1, v);
        }
        float un[NLMAX], qn[NNMAX][ND], ubn[NLMAX];
#pragma unroll
        for (int L = 0; L < NLMAX; ++L) un[L] = ubn[L] = ua[L];   // defined when !has_next
        // labels of plane z + 1 (owned when z + 1 < ze, else the halo plane)
        if (va && has_next) {
            float qz[NNMAX];
#pragma unroll
            for (int A = 0; A < NNMAX; ++A) qz[A] = qa[A][ND - 1];
            label_point<ND, NLMAX, NNMAX, IDENT, T>(a, b, xa, ya, z + 1, qz, own && z + 1 < ze,
                                                    un, qn);
        }
        if (vb && has_next) {
            float qz[NNMAX];
#pragma unroll
            for (int A = 0; A < NNMAX; ++A) qz[A] = qb[A][ND - 1];
            label_point<ND, NLMAX, NNMAX, IDENT, T>(a, b, xb, yb, z + 1, qz, false, ubn, qb);
        }
        // flow step of the owned voxels of plane z
        if (own) {
            const int v = (z * a.ny + ya) * a.nx + xa;
            const bool h[3] = {xa < a.nx - 1, ya < a.ny - 1, ND == 3 && has_next};
            float gu[NLMAX][ND];
#pragma unroll
            for (int L = 0; L < NLMAX; ++L) {
                gu[L][0] = h[0] ? lds[L][row][col + 1] - ua[L] : 0.f;
                gu[L][1] = h[1] ? lds[L][row + 1][col] - ua[L] : 0.f;
                if constexpr (ND == 3) gu[L][2] = h[2] ? un[L] - ua[L] : 0.f;
            }
#pragma unroll
            for (int A = 0; A < NNMAX; A += 2) {
                if (A < a.nn) {
                    float p[2][ND];
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
#pragma unroll
                        for (int k = 0; k < ND; ++k) p[j][k] = 0.f;
                        if (A + j < a.nn) {
                            float G[3];
                            grad_U<ND, NLMAX, IDENT>(a, A + j, gu, G);
                            flow_project<ND>(a, qa[A + j], G, h, sv[A + j], p[j]);
                        }
                    }
#pragma unroll
                    for (int k = 0; k < ND; ++k)
                        st_q2<T, ND>(a.q_out, b, a.nn, A, k, V, (unsigned)v, p[0][k], p[1][k]);
                }
            }
        }
        __syncthreads();   // plane z of the LDS is no longer read
        if (has_next) {
            if (va) {
#pragma unroll
                for (int L = 0; L < NLMAX; ++L) {
                    lds[L][row][col] = un[L];
                    ua[L] = un[L];
                }
#pragma unroll
                for (int A = 0; A < NNMAX; ++A)
#pragma unroll
                    for (int k = 0; k < ND; ++k) qa[A][k] = qn[A][k];
            }
            if (vb) {
#pragma unroll
                for (int L = 0; L < NLMAX; ++L) lds[L][col][FTX] = ubn[L];
            }
        }
        __syncthreads();
    }
}

template <int ND, typename T, typename F>
hipError_t fused_bucket(bool ident, int nl, int nn, F &f) {
    if (ident) {
        if (nl <= 4) return f.template operator()<ND, 4, 4, true, T>();
        if (nl <= 8) return f.template operator()<ND, 8, 8, true, T>();
        return f.template operator()<ND, 16, 16, true, T>();
    }
    if (nl <= 4 && nn <= 8) return f.template operator()<ND, 4, 8, false, T>();
    if (nl <= 8 && nn <= 16) return f.template operator()<ND, 8, 16, false, T>();
    return f.template operator()<ND, 16, 16, false, T>();
}

template <typename F>
hipError_t fused_dispatch(int nd, int storage, bool ident, int nl, int nn, F &&f) {
    if (nd == 2) {
        if (storage == PF_BF16) return fused_bucket<2, bf16s>(ident, nl, nn, f);
        if (storage == PF_FP16) return fused_bucket<2, f16s>(ident, nl, nn, f);
        return fused_bucket<2, float>(ident, nl, nn, f);
    }
    if (storage == PF_BF16) return fused_bucket<3, bf16s>(ident, nl, nn, f);
    if (storage == PF_FP16) return fused_bucket<3, f16s>(ident, nl, nn, f);
    return fused_bucket<3, float>(ident, nl, nn, f);
}

}  // namespace

bool fused_supported(int nd, int nl, int nn, bool identity) {
    (void)nd;
    if (identity) return nl <= 16;
    return nl <= 16 && nn <= 16;
}

// PF_KERNEL_AUTO: the fused single pass where it measured faster than the
// two-pass kernels on MI355X (3-D Potts with float32 state); the two-pass
// kernels elsewhere (their lower register pressure wins for 16-bit state and
// for label graphs).
bool fused_preferred(int nd, int nl, int nn, bool identity, int storage) {
    return identity && nd == 3 && storage == PF_FP32 && fused_supported(nd, nl, nn, identity);
}

FusedGeom fused_geometry(const StepArgs &a) { return tile_geometry(a, FTX, FTY); }

FusedGeom tile_geometry(const StepArgs &a, int width, int rows) {
    FusedGeom g{};
    g.tiles_x = (a.nx + width - 1) / width;
    g.tiles_y = (a.ny + rows - 1) / rows;
    const long tiles = (long)g.tiles_x * g.tiles_y * a.B;
    // aim for about two resident blocks per compute unit on 256 CUs, with
    // chunks of at least 16 planes (each chunk recomputes one extra plane)
    const long target = 512;
    long chunks = (target + tiles - 1) / tiles;
    const long max_chunks = (a.nz + 15) / 16;
    if (chunks > max_chunks) chunks = max_chunks;
    if (chunks < 1) chunks = 1;
    g.cz = (int)((a.nz + chunks - 1) / chunks);
    g.n_chunks = (a.nz + g.cz - 1) / g.cz;
    g.blocks = tiles * g.n_chunks;
    return g;
}

hipError_t launch_fused(const StepArgs &a, bool ident, int nd, int storage, hipStream_t s) {
    const FusedGeom g = fused_geometry(a);
    if (g.blocks <= 0 || g.blocks > 0x7fffffffL) return hipErrorInvalidValue;
    return fused_dispatch(nd, storage, ident, a.nl, a.nn,
                          [&]<int ND, int NL, int NN, bool ID, typename T>() {
                              k_fused<ND, NL, NN, ID, T>
                                  <<<(unsigned)g.blocks, FTHREADS, 0, s>>>(a, g);
                              return hipGetLastError();
                          });
}

}  // namespace pf
