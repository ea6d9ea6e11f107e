// Reverse-mode kernels of the unrolled pseudo-flow iteration (float32 state),
// for gradients of a loss on the final log-labels with respect to the data
// terms D and the capacities S.
//
// Forward step k (path-weight form, any label graph; Potts is W = identity):
//   d = D + W^T div q_k,  ell_{k+1} = t - LSE(t),  t = ell_k - d / c,
//   u' = exp(ell_{k+1}),  U = W u',  p = q_k - c tau grad U (zero on the last
//   index of each axis),  q_{k+1} = p min(1, S / |p|).
// Reverse step k, given lbar = dLoss/dt^{(k+1)} (the gradient that reached the
// label step of step k+1; for the last step the loss gradient on ell_K) and
// pbar = dLoss/dp^{(k+1)}:
//   KA: qbar_{k+1} = pbar^{(k+1)} + grad(W lbar) / c        (through p and div)
//       pbar^{(k)} = J_Proj(p)^T qbar_{k+1},  Sbar += (p . qbar) / |p| if |p| > S
//   KB: Ubar = c tau div pbar^{(k)},  g = lbar + (W^T Ubar) * u'   (total dLoss/dell_{k+1})
//       lbar <- g - u' sum_L g_L,  Dbar -= lbar / c
// KA at x reads lbar at x and x + e_k; KB at x reads the new pbar at x and
// x - e_k.  Two variants:
//   * two kernels (KA, then KB), each updating its buffer in place (a thread
//     writes only its own voxel);
//   * one fused kernel: a block owns an RTX x RTY tile of (x, y) columns and
//     marches a chunk of z planes; the new pbar of the plane is exchanged
//     through LDS, the points one row / one column before the tile are
//     recomputed by two extra halo wavefronts, and along z the backward
//     neighbour is the thread's own previous plane.  lbar and pbar are read
//     from one buffer and written to another, since the halo points read
//     values that the neighbouring blocks overwrite.  In 2-D (rows of up to
//     512 voxels) a block instead spans whole rows and marches along y, with
//     no halo points (k_adj_rows).
// Both variants evaluate the same per-point expressions (ka_point, kb_point)
// and give the same gradients bit for bit.

#include <hip/hip_runtime.h>
#include <math.h>

#include "pf_device.h"
#include "pf_internal.h"

namespace pf {
namespace {

using namespace dev;

constexpr int RTX = 64;               // tile width = one wavefront
constexpr int RTY = 8;                // owned rows per tile (the fused forward tile)
constexpr int RTHREADS = RTX * (RTY + 2);   // owned rows + two halo wavefronts

// KA at voxel c (index uv) of problem b: the new pbar (out, 0 on the last
// index of each axis and for padding flows), the capacity-gradient
// contributions (sb) and the new log-labels and incoming lbar at the voxel
// (e0, l0, which KB needs).  All loads are issued first, unconditionally
// (clamped indices stay in bounds).
template <int ND, int NLMAX, int NNMAX, bool IDENT>
__device__ __forceinline__ void ka_point(const StepArgs &a, const AdjArgs &g, int b,
                                         const Coord &c, unsigned uv, float (&out)[NNMAX][ND],
                                         float (&sb)[NNMAX], float (&e0)[NLMAX],
                                         float (&l0)[NLMAX]) {
    const size_t V = (size_t)a.V;
    const bool h[3] = {c.x < a.nx - 1, c.y < a.ny - 1, ND == 3 && c.z < a.nz - 1};
    const int off[3] = {h[0] ? 1 : 0, h[1] ? a.nx : 0, h[2] ? a.nx * a.ny : 0};

    float en[NLMAX][ND], lnb[NLMAX][ND];
    float qv[NNMAX][ND], pb[NNMAX][ND], sv[NNMAX];
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        const int Lc = L < a.nl ? L : a.nl - 1;
        const float *el = field<float>(g.ell_next, b, a.nl, Lc, V);
        const float *lb = field<float>(g.lbar_in, b, a.nl, Lc, V);
        e0[L] = ldf(el, uv);
        l0[L] = ldf(lb, uv);
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            en[L][k] = ldf(el, uv + (unsigned)off[k]);
            lnb[L][k] = ldf(lb, uv + (unsigned)off[k]);
        }
    }
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) {
        const int Ac = A < a.nn ? A : a.nn - 1;
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            qv[A][k] = ldf(field<float>(g.q_k, b, a.nn * ND, Ac * ND + k, V), uv);
            pb[A][k] = ldf(field<float>(g.pbar_in, b, a.nn * ND, Ac * ND + k, V), uv);
        }
        sv[A] = smooth(a, b, Ac, (int)uv);
    }
    // forward quantities (grad u', grad U, p) and grad lbar
    float gu[NLMAX][ND], gl[NLMAX][ND];
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        const float u0 = __expf(e0[L]);
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            gu[L][k] = h[k] ? __expf(en[L][k]) - u0 : 0.f;
            gl[L][k] = h[k] ? lnb[L][k] - l0[L] : 0.f;
        }
    }
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) {
        float G[3], GL[3], p[ND], qb[ND];
        grad_U<ND, NLMAX, IDENT>(a, A, gu, G);
        grad_U<ND, NLMAX, IDENT>(a, A, gl, GL);       // grad (W lbar)
        float n2 = 0.f, dot = 0.f;
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            p[k] = h[k] ? fmaf(-a.ctau, G[k], qv[A][k]) : 0.f;
            qb[k] = g.first ? 0.f : (h[k] ? pb[A][k] + GL[k] * a.inv_c : 0.f);
            n2 = fmaf(p[k], p[k], n2);
            dot = fmaf(p[k], qb[k], dot);
        }
        const float S = sv[A];
        float s = 0.f;
        if (n2 > S * S) {
            const float rn = rsqrtf(n2);
            const float sc = S * rn;
            const float proj = dot / n2;
#pragma unroll
            for (int k = 0; k < ND; ++k) out[A][k] = sc * (qb[k] - proj * p[k]);
            s = dot * rn;
        } else {
#pragma unroll
            for (int k = 0; k < ND; ++k) out[A][k] = qb[k];
        }
        const bool live = A < a.nn;
#pragma unroll
        for (int k = 0; k < ND; ++k) out[A][k] = (live && h[k]) ? out[A][k] : 0.f;
        sb[A] = live ? s : 0.f;
    }
}

// KB at one voxel: e, lb = new log-labels and incoming lbar at the voxel,
// p0 / pm = new pbar at x / at x - e_k.  Returns the new lbar (tb).
template <int ND, int NLMAX, int NNMAX, bool IDENT>
__device__ __forceinline__ void kb_point(const StepArgs &a, const float (&e)[NLMAX],
                                         const float (&lb)[NLMAX], const float (&p0)[NNMAX][3],
                                         const float (&pm)[NNMAX][3], const bool (&fwd)[3],
                                         const bool (&bwd)[3], float (&tb)[NLMAX]) {
    // ubar_L = sum_A W[A][L] * c tau div pbar_A
    float ub[NLMAX];
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) ub[L] = 0.f;
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) {
        const float dv = a.ctau * div_from<ND>(p0[A], pm[A], fwd, bwd);
        if constexpr (IDENT) {
            ub[A] += dv;
        } else {
#pragma unroll
            for (int L = 0; L < NLMAX; ++L) ub[L] = fmaf(wgt(a, A, L), dv, ub[L]);
        }
    }
    // adjoint of ell_{k+1} = t - LSE(t): tbar = gtot - u' sum(gtot)
    float gt[NLMAX], u[NLMAX], sg = 0.f;
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        u[L] = __expf(e[L]);
        gt[L] = L < a.nl ? fmaf(ub[L], u[L], lb[L]) : 0.f;
        sg += gt[L];
    }
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) tb[L] = gt[L] - u[L] * sg;
}

// Capacity-gradient accumulator of one voxel: one field summed over the
// flows when every flow shares one capacity field, else one value per flow.
// Loaded ahead (with the other loads of the point), updated by add_sbar.
template <int NNMAX>
__device__ __forceinline__ void load_sbar(const StepArgs &a, const AdjArgs &g, int b, unsigned uv,
                                          float (&acc)[NNMAX]) {
    const size_t V = (size_t)a.V;
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) {
        const int f = g.sbar_shared ? 0 : (A < a.nn ? A : a.nn - 1);
        acc[A] = ldf(field<float>(g.sbar, b, g.sbar_shared ? 1 : a.nn, f, V), uv);
    }
}

template <int NNMAX>
__device__ __forceinline__ void add_sbar(const StepArgs &a, const AdjArgs &g, int b, unsigned uv,
                                         const float (&acc)[NNMAX], const float (&sb)[NNMAX]) {
    const size_t V = (size_t)a.V;
    if (g.sbar_shared) {
        float s = 0.f;
#pragma unroll
        for (int A = 0; A < NNMAX; ++A) s += sb[A];
        sto(field_w<float>(g.sbar, b, 1, 0, V), uv, acc[0] + s);
    } else {
#pragma unroll
        for (int A = 0; A < NNMAX; ++A)
            if (A < a.nn) sto(field_w<float>(g.sbar, b, a.nn, A, V), uv, acc[A] + sb[A]);
    }
}

// D-gradient accumulator of one voxel, loaded ahead.
template <int NLMAX>
__device__ __forceinline__ void load_dbar(const StepArgs &a, const AdjArgs &g, int b, unsigned uv,
                                          float (&acc)[NLMAX]) {
    const size_t V = (size_t)a.V;
#pragma unroll
    for (int L = 0; L < NLMAX; ++L)
        acc[L] = ldf(field<float>(g.dbar, b, a.nl, L < a.nl ? L : a.nl - 1, V), uv);
}

// Stores of KB at an owned voxel: the new lbar, and D's gradient -= lbar / c.
template <int NLMAX>
__device__ __forceinline__ void store_label_adjoint(const StepArgs &a, const AdjArgs &g, int b,
                                                    unsigned uv, const float (&dacc)[NLMAX],
                                                    const float (&tb)[NLMAX]) {
    const size_t V = (size_t)a.V;
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        if (L < a.nl) {
            sto(field_w<float>(g.lbar_out, b, a.nl, L, V), uv, tb[L]);
            sto(field_w<float>(g.dbar, b, a.nl, L, V), uv, dacc[L] - tb[L] * a.inv_c);
        }
    }
}

// ------------------------------------------------------ two kernels ------

template <int ND, int NLMAX, int NNMAX, bool IDENT>
__global__ __launch_bounds__(kBlock) void k_adj_flow(StepArgs a, AdjArgs g) {
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= a.V) return;
    const int b = blockIdx.y;
    const Coord c = coord_of(v, a.nx, a.ny);
    const unsigned uv = (unsigned)v;
    const size_t V = (size_t)a.V;
    float out[NNMAX][ND], sb[NNMAX], e0[NLMAX], l0[NLMAX], sacc[NNMAX];
    load_sbar<NNMAX>(a, g, b, uv, sacc);
    ka_point<ND, NLMAX, NNMAX, IDENT>(a, g, b, c, uv, out, sb, e0, l0);
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) {
        if (A < a.nn) {
#pragma unroll
            for (int k = 0; k < ND; ++k)
                sto(field_w<float>(g.pbar_out, b, a.nn * ND, A * ND + k, V), uv, out[A][k]);
        }
    }
    add_sbar<NNMAX>(a, g, b, uv, sacc, sb);
}

template <int ND, int NLMAX, int NNMAX, bool IDENT>
__global__ __launch_bounds__(kBlock) void k_adj_label(StepArgs a, AdjArgs g) {
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= a.V) return;
    const int b = blockIdx.y;
    const Coord c = coord_of(v, a.nx, a.ny);
    const size_t V = (size_t)a.V;
    const unsigned uv = (unsigned)v;
    int m[3];
    bool bwd[3];
    backward_offsets(c, a, m, bwd);
    const bool fwd[3] = {c.x < a.nx - 1, c.y < a.ny - 1, ND == 3 && c.z < a.nz - 1};

    float e[NLMAX], lb[NLMAX], dacc[NLMAX], p0[NNMAX][3], pm[NNMAX][3];
    load_dbar<NLMAX>(a, g, b, uv, dacc);
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        const int Lc = L < a.nl ? L : a.nl - 1;
        e[L] = ldf(field<float>(g.ell_next, b, a.nl, Lc, V), uv);
        lb[L] = ldf(field<float>(g.lbar_in, b, a.nl, Lc, V), uv);
    }
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) {
        const int Ac = A < a.nn ? A : a.nn - 1;
#pragma unroll
        for (int k = 0; k < 3; ++k) p0[A][k] = pm[A][k] = 0.f;
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            const float *pk = field<float>(g.pbar_out, b, a.nn * ND, Ac * ND + k, V);
            p0[A][k] = ldf(pk, uv);
            pm[A][k] = ldf(pk, uv - (unsigned)m[k]);
        }
    }
    float tb[NLMAX];
    kb_point<ND, NLMAX, NNMAX, IDENT>(a, e, lb, p0, pm, fwd, bwd, tb);
    store_label_adjoint<NLMAX>(a, g, b, uv, dacc, tb);
}

// ------------------------------------------------------ fused kernel -----

template <int ND, int NLMAX, int NNMAX, bool IDENT>
__global__ __launch_bounds__(RTHREADS) void k_adj_fused(StepArgs a, AdjArgs g, FusedGeom geo) {
    // new pbar of the current plane: x components (column 0 = x0 - 1) and
    // y components (row 0 = y0 - 1)
    __shared__ float sx[NNMAX][RTY][RTX + 1];
    __shared__ float sy[NNMAX][RTY + 1][RTX];
    const int wave = threadIdx.x / RTX;
    const int lane = threadIdx.x % RTX;

    // XCD-aware block -> tile mapping (as in the fused forward kernel)
    const int nb = gridDim.x;
    const int pblk = blockIdx.x;
    const int lblk = (nb % 8 == 0) ? (pblk % 8) * (nb / 8) + pblk / 8 : pblk;
    const int bx = lblk % geo.tiles_x;
    int r = lblk / geo.tiles_x;
    const int by = r % geo.tiles_y;
    r /= geo.tiles_y;
    const int ch = r % geo.n_chunks;
    const int b = r / geo.n_chunks;
    const int x0 = bx * RTX, y0 = by * RTY;
    const int zs = ch * geo.cz;
    const int ze = min(a.nz, zs + geo.cz);
    const size_t V = (size_t)a.V;

    // point A: owned voxel column (waves 0 .. RTY-1), or the row before the
    // tile (wave RTY); point B (wave RTY+1): the column before the tile
    const int xa = x0 + lane, ya = wave == RTY ? y0 - 1 : y0 + wave;
    const bool va = wave <= RTY && xa < a.nx && ya >= 0 && ya < a.ny;
    const bool own = wave < RTY && va;
    const int xb = x0 - 1, yb = y0 + lane;
    const bool vb = wave == RTY + 1 && lane < RTY && xb >= 0 && yb < a.ny;

    float pz[NNMAX];                 // new pbar_z one plane below (owned points)
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) pz[A] = 0.f;
    if (ND == 3 && own && zs > 0) {
        float out[NNMAX][ND], sb[NNMAX], e0[NLMAX], l0[NLMAX];
        ka_point<ND, NLMAX, NNMAX, IDENT>(a, g, b, Coord{xa, ya, zs - 1},
                                          (unsigned)(((zs - 1) * a.ny + ya) * a.nx + xa), out, sb,
                                          e0, l0);
#pragma unroll
        for (int A = 0; A < NNMAX; ++A) pz[A] = out[A][ND - 1];
    }

    for (int z = zs; z < ze; ++z) {
        float out[NNMAX][ND], sb[NNMAX], e0[NLMAX], l0[NLMAX], dacc[NLMAX], sacc[NNMAX];
        const unsigned uva = (unsigned)((z * a.ny + ya) * a.nx + xa);
        if (own) {
            load_dbar<NLMAX>(a, g, b, uva, dacc);
            load_sbar<NNMAX>(a, g, b, uva, sacc);
        }
        if (va) {
            ka_point<ND, NLMAX, NNMAX, IDENT>(a, g, b, Coord{xa, ya, z}, uva, out, sb, e0, l0);
            if (own) {
#pragma unroll
                for (int A = 0; A < NNMAX; ++A) {
                    sx[A][wave][lane + 1] = out[A][0];
                    sy[A][wave + 1][lane] = out[A][1];
                }
            } else {
#pragma unroll
                for (int A = 0; A < NNMAX; ++A) sy[A][0][lane] = out[A][1];
            }
        }
        if (vb) {
            float ob[NNMAX][ND], sbb[NNMAX], eb[NLMAX], lbb[NLMAX];
            ka_point<ND, NLMAX, NNMAX, IDENT>(a, g, b, Coord{xb, yb, z},
                                              (unsigned)((z * a.ny + yb) * a.nx + xb), ob, sbb, eb,
                                              lbb);
#pragma unroll
            for (int A = 0; A < NNMAX; ++A) sx[A][lane][0] = ob[A][0];
        }
        __syncthreads();
        if (own) {
            const bool fwd[3] = {xa < a.nx - 1, ya < a.ny - 1, ND == 3 && z < a.nz - 1};
            const bool bwd[3] = {xa > 0, ya > 0, ND == 3 && z > 0};
            float p0[NNMAX][3], pm[NNMAX][3];
#pragma unroll
            for (int A = 0; A < NNMAX; ++A) {
                p0[A][0] = out[A][0];
                p0[A][1] = out[A][1];
                p0[A][2] = ND == 3 ? out[A][ND - 1] : 0.f;
                pm[A][0] = sx[A][wave][lane];
                pm[A][1] = sy[A][wave][lane];
                pm[A][2] = pz[A];
            }
            float tb[NLMAX];
            kb_point<ND, NLMAX, NNMAX, IDENT>(a, e0, l0, p0, pm, fwd, bwd, tb);
            store_label_adjoint<NLMAX>(a, g, b, uva, dacc, tb);
#pragma unroll
            for (int A = 0; A < NNMAX; ++A) {
                if (A < a.nn) {
#pragma unroll
                    for (int k = 0; k < ND; ++k)
                        sto(field_w<float>(g.pbar_out, b, a.nn * ND, A * ND + k, V), uva, out[A][k]);
                }
                pz[A] = p0[A][2];
            }
            add_sbar<NNMAX>(a, g, b, uva, sacc, sb);
        }
        __syncthreads();
    }
}

// ------------------------------------------------- 2-D row march ---------

// In 2-D the fused kernel above has no planes to march and spends two halo
// wavefronts per 8-row tile.  Here a block spans every column of a problem
// (one thread per column, one wavefront per 64 columns) and marches a chunk
// of rows: KB at (x, y) takes the new pbar_x at x - 1 from its neighbour
// thread through LDS (by row parity, one barrier per row) and the new pbar_y
// at y - 1 from the thread's own previous row, so no point is computed twice
// except KA on the row before a chunk.
constexpr int ROW_COLS = 512;         // widest row a block spans

template <int NLMAX, int NNMAX, bool IDENT>
__global__ __launch_bounds__(ROW_COLS) void k_adj_rows(StepArgs a, AdjArgs g, int cy, int n_chunks) {
    __shared__ float xs[2][NNMAX][ROW_COLS];       // new pbar_x of the row, by row parity
    const int x = threadIdx.x;
    const int ch = blockIdx.x % n_chunks;
    const int b = blockIdx.x / n_chunks;
    const bool vx = x < a.nx;
    const int ys = ch * cy;
    const int ye = min(a.ny, ys + cy);
    const size_t V = (size_t)a.V;

    float py[NNMAX];                 // new pbar_y on the row below
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) py[A] = 0.f;
    if (vx && ys > 0) {
        float out[NNMAX][2], sb[NNMAX], e0[NLMAX], l0[NLMAX];
        ka_point<2, NLMAX, NNMAX, IDENT>(a, g, b, Coord{x, ys - 1, 0},
                                         (unsigned)((ys - 1) * a.nx + x), out, sb, e0, l0);
#pragma unroll
        for (int A = 0; A < NNMAX; ++A) py[A] = out[A][1];
    }

    for (int y = ys; y < ye; ++y) {
        const int par = y & 1;
        float out[NNMAX][2], sb[NNMAX], e0[NLMAX], l0[NLMAX], dacc[NLMAX], sacc[NNMAX];
        const unsigned uv = (unsigned)(y * a.nx + x);
        if (vx) {
            load_dbar<NLMAX>(a, g, b, uv, dacc);
            load_sbar<NNMAX>(a, g, b, uv, sacc);
            ka_point<2, NLMAX, NNMAX, IDENT>(a, g, b, Coord{x, y, 0}, uv, out, sb, e0, l0);
#pragma unroll
            for (int A = 0; A < NNMAX; ++A) xs[par][A][x] = out[A][0];
        }
        __syncthreads();   // the row's new pbar_x is in LDS
        if (vx) {
            const bool fwd[3] = {x < a.nx - 1, y < a.ny - 1, false};
            const bool bwd[3] = {x > 0, y > 0, false};
            float p0[NNMAX][3], pm[NNMAX][3];
#pragma unroll
            for (int A = 0; A < NNMAX; ++A) {
                p0[A][0] = out[A][0];
                p0[A][1] = out[A][1];
                p0[A][2] = 0.f;
                pm[A][0] = x > 0 ? xs[par][A][x - 1] : 0.f;
                pm[A][1] = py[A];
                pm[A][2] = 0.f;
            }
            float tb[NLMAX];
            kb_point<2, NLMAX, NNMAX, IDENT>(a, e0, l0, p0, pm, fwd, bwd, tb);
            store_label_adjoint<NLMAX>(a, g, b, uv, dacc, tb);
#pragma unroll
            for (int A = 0; A < NNMAX; ++A) {
                if (A < a.nn) {
                    sto(field_w<float>(g.pbar_out, b, a.nn * 2, A * 2, V), uv, out[A][0]);
                    sto(field_w<float>(g.pbar_out, b, a.nn * 2, A * 2 + 1, V), uv, out[A][1]);
                }
                py[A] = out[A][1];
            }
            add_sbar<NNMAX>(a, g, b, uv, sacc, sb);
        }
    }
}

// ------------------------------------------------------ utilities --------

__global__ __launch_bounds__(kBlock) void k_fill(float *p, size_t n, float val) {
    const size_t stride = (size_t)gridDim.x * kBlock;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) p[i] = val;
}

__global__ __launch_bounds__(kBlock) void k_copy_f(const float *__restrict__ a, float *__restrict__ b,
                                                   size_t n) {
    const size_t stride = (size_t)gridDim.x * kBlock;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

// dS for a per-node constant: sum over problems and voxels, fp64, fixed order.
__global__ __launch_bounds__(kBlock) void k_sum_nodes(const float *sbar, int B, int nn, size_t V,
                                                      float *out) {
    __shared__ double red[kBlock];
    const int A = blockIdx.x;
    double s = 0.0;
    for (int b = 0; b < B; ++b) {
        const float *p = sbar + ((size_t)b * nn + A) * V;
        for (size_t i = threadIdx.x; i < V; i += kBlock) s += (double)p[i];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[A] = (float)red[0];
}

unsigned sblocks(size_t n) {
    const size_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < 4096 ? (b ? b : 1) : 4096);
}

template <typename F>
hipError_t adj_dispatch(int nd, bool ident, int nl, int nn, F &&f) {
    auto by = [&]<int ND>() -> hipError_t {
        if (ident) {
            if (nl <= 4) return f.template operator()<ND, 4, 4, true>();
            if (nl <= 8) return f.template operator()<ND, 8, 8, true>();
            return f.template operator()<ND, 16, 16, true>();
        }
        if (nl <= 4 && nn <= 8) return f.template operator()<ND, 4, 8, false>();
        if (nl <= 8 && nn <= 16) return f.template operator()<ND, 8, 16, false>();
        if (nn <= 16) return f.template operator()<ND, 16, 16, false>();
        return f.template operator()<ND, 16, 32, false>();
    };
    return nd == 2 ? by.template operator()<2>() : by.template operator()<3>();
}

// The fused reverse kernel keeps a point's whole adjoint state in registers;
// it is built for the buckets that fit in the register budget of a
// 640-thread block without spilling: Potts up to 8
// labels in 2-D (builds of 4, 6 and 8) and 4 in 3-D, label graphs up to 4
// leaves / 8 flows in 2-D.
template <typename F>
hipError_t adj_fused_dispatch(int nd, bool ident, int nl, F &&f) {
    if (nd == 2) {
        if (!ident) return f.template operator()<2, 4, 8, false>();
        if (nl <= 4) return f.template operator()<2, 4, 4, true>();
        if (nl <= 6) return f.template operator()<2, 6, 6, true>();
        return f.template operator()<2, 8, 8, true>();
    }
    return f.template operator()<3, 4, 4, true>();
}

}  // namespace

bool adj_fused_supported(int nd, int nl, int nn, bool identity) {
    if (nd == 2) return identity ? nl <= 8 : (nl <= 4 && nn <= 8);
    if (nd == 3) return identity && nl <= 4;
    return false;
}

// PF_KERNEL_AUTO takes the fused reverse step where it runs as the row march
// (2-D rows of up to 512 voxels): the differentiation batch's backward 9.07
// (6-label build) against 10.0 ms with the two kernels.  The tile form (3-D, wider rows)
// measured slower than the two kernels and is used only on request.
bool adj_fused_preferred(int nd, int nx, int nl, int nn, bool identity) {
    return nd == 2 && nx <= ROW_COLS && adj_fused_supported(nd, nl, nn, identity);
}

hipError_t launch_adj_flow(const StepArgs &a, const AdjArgs &g, bool ident, int nd, hipStream_t s) {
    const dim3 grid((unsigned)((a.V + kBlock - 1) / kBlock), (unsigned)a.B, 1);
    return adj_dispatch(nd, ident, a.nl, a.nn, [&]<int ND, int NL, int NN, bool ID>() {
        k_adj_flow<ND, NL, NN, ID><<<grid, kBlock, 0, s>>>(a, g);
        return hipGetLastError();
    });
}

hipError_t launch_adj_label(const StepArgs &a, const AdjArgs &g, bool ident, int nd, hipStream_t s) {
    const dim3 grid((unsigned)((a.V + kBlock - 1) / kBlock), (unsigned)a.B, 1);
    return adj_dispatch(nd, ident, a.nl, a.nn, [&]<int ND, int NL, int NN, bool ID>() {
        k_adj_label<ND, NL, NN, ID><<<grid, kBlock, 0, s>>>(a, g);
        return hipGetLastError();
    });
}

hipError_t launch_adj_fused(const StepArgs &a, const AdjArgs &g, bool ident, int nd, hipStream_t s) {
    if (!adj_fused_supported(nd, a.nl, a.nn, ident)) return hipErrorInvalidValue;
    if (nd == 2 && a.nx <= ROW_COLS) {
        // chunks of at least 4 rows; about 4096 wavefronts over the launch
        // (16 per compute unit: on the 16 x 256^2 differentiation batch 8 and
        // 16 rows per chunk measured 1-2% slower, 2 and 1 row 5-20% slower)
        const long waves = (long)a.B * ((a.nx + 63) / 64);
        const long want = (4096 + waves - 1) / waves;
        const long max_chunks = (a.ny + 3) / 4;
        const int n0 = (int)(want < max_chunks ? want : max_chunks);
        const int cy = (a.ny + n0 - 1) / n0;
        const int n_chunks = (a.ny + cy - 1) / cy;
        const long blocks = (long)a.B * n_chunks;
        if (blocks <= 0 || blocks > 0x7fffffffL) return hipErrorInvalidValue;
        const unsigned threads = (unsigned)((a.nx + 63) / 64 * 64);
        return adj_fused_dispatch(nd, ident, a.nl, [&]<int ND, int NL, int NN, bool ID>() {
            k_adj_rows<NL, NN, ID><<<(unsigned)blocks, threads, 0, s>>>(a, g, cy, n_chunks);
            return hipGetLastError();
        });
    }
    const FusedGeom geo = tile_geometry(a, RTX, RTY);
    if (geo.blocks <= 0 || geo.blocks > 0x7fffffffL) return hipErrorInvalidValue;
    return adj_fused_dispatch(nd, ident, a.nl, [&]<int ND, int NL, int NN, bool ID>() {
        k_adj_fused<ND, NL, NN, ID><<<(unsigned)geo.blocks, RTHREADS, 0, s>>>(a, g, geo);
        return hipGetLastError();
    });
}

hipError_t launch_fill(float *p, size_t n, float val, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_fill<<<sblocks(n), kBlock, 0, s>>>(p, n, val);
    return hipGetLastError();
}

hipError_t launch_copy_f(const float *a, float *b, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_copy_f<<<sblocks(n), kBlock, 0, s>>>(a, b, n);
    return hipGetLastError();
}

hipError_t launch_sum_nodes(const float *sbar, int B, int nn, size_t V, float *out, hipStream_t s) {
    if (nn < 1) return hipErrorInvalidValue;
    k_sum_nodes<<<nn, kBlock, 0, s>>>(sbar, B, nn, V, out);
    return hipGetLastError();
}

}  // namespace pf
