// gfx950 kernels of the pseudo-flow continuous max-flow iteration.
//
// One iteration (Algorithm 1 for Potts, Algorithm 2 for DAGMF/HMF,
// Algorithm 3 for the Ishikawa chain) in path-weight form:
//   label pass:  d_L = D_L + sum_A W[A][L] div q_A           (top-down excess)
//                ell_L <- ell_L - d_L/c - LSE_L'(ell_L' - d_L'/c)   (proximal step)
//   flow pass:   grad U_A = sum_L W[A][L] grad u_L,  u = exp(ell)  (bottom-up labels)
//                q_A <- Proj_{|q_A| <= S_A}(q_A - c tau grad U_A)  (Chambolle step)
// Potts is W = identity and is compiled as its own specialisation.
//
// State is stored as ell = ln u (float32, bfloat16 or float16) and flows in
// the same type; all arithmetic is float32; energy/dual reductions are float64.
// The path is HBM-bandwidth bound (about one flop per byte), so there is no
// matrix-core work: one voxel per lane, x fastest, every field read and
// written with unit stride across the wavefront.

#include <hip/hip_runtime.h>
#include <math.h>

#include "pf_device.h"
#include "pf_internal.h"

namespace pf {
namespace {

using namespace dev;

// --------------------------------------------------------- label pass ----

template <int ND, int NLMAX, int NNMAX, bool IDENT, typename T>
__device__ __forceinline__ void label_body(const StepArgs &a) {
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= a.V) return;
    const int b = blockIdx.y;
    const Coord c = coord_of(v, a.nx, a.ny);
    const size_t V = (size_t)a.V;
    int m[3];
    bool bwd[3];
    backward_offsets(c, a, m, bwd);
    const bool fwd[3] = {c.x < a.nx - 1, c.y < a.ny - 1, ND == 3 && c.z < a.nz - 1};

    // load phase: every load unconditional, indices clamped into the volume
    // and into the label / node ranges; uniform field bases + 32-bit offsets
    const unsigned uv = (unsigned)v;
    float d[NLMAX], e[NLMAX], q0[NNMAX][3], qm[NNMAX][3];
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        const int Lc = L < a.nl ? L : a.nl - 1;
        d[L] = ldf(field<float>(a.D, b, a.nl, Lc, V), uv);
        e[L] = ld_ell<T>(a.ell_in, b, a.nl, L, V, uv);
    }
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) {
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            q0[A][k] = ld_q<T, ND>(a.q_in, b, a.nn, A, k, V, uv);
            qm[A][k] = ld_q<T, ND>(a.q_in, b, a.nn, A, k, V, uv - (unsigned)m[k]);
        }
    }
    // compute phase
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) add_excess<NLMAX, IDENT>(a, d, A, div_from<ND>(q0[A], qm[A], fwd, bwd));
    entropic_step<NLMAX>(a, d, e);
#pragma unroll
    for (int L = 0; L < NLMAX; L += 2) st_ell2<T>(a.ell_out, b, a.nl, L, V, uv, e[L], e[L + 1]);
}

template <int ND, int NLMAX, int NNMAX, bool IDENT, typename T>
__global__ __launch_bounds__(kBlock) void k_label(StepArgs a) {
    label_body<ND, NLMAX, NNMAX, IDENT, T>(a);
}

// ---------------------------------------------------------- flow pass ----

template <int ND, int NLMAX, int NNMAX, bool IDENT, typename T>
__device__ __forceinline__ void flow_body(const StepArgs &a) {
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= a.V) return;
    const int b = blockIdx.y;
    const Coord c = coord_of(v, a.nx, a.ny);
    const size_t V = (size_t)a.V;
    const bool h[3] = {c.x < a.nx - 1, c.y < a.ny - 1, ND == 3 && c.z < a.nz - 1};
    // forward offsets, 0 on the last index so that the loads stay in the volume
    const int off[3] = {h[0] ? 1 : 0, h[1] ? a.nx : 0, h[2] ? a.nx * a.ny : 0};

    // load phase (uniform field bases + 32-bit lane offsets)
    const unsigned uv = (unsigned)v;
    float e0[NLMAX], en[NLMAX][ND], qv[NNMAX][ND], sv[NNMAX];
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        e0[L] = ld_ell<T>(a.ell_in, b, a.nl, L, V, uv);
#pragma unroll
        for (int k = 0; k < ND; ++k) en[L][k] = ld_ell<T>(a.ell_in, b, a.nl, L, V, uv + (unsigned)off[k]);
    }
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) {
        const int Ac = A < a.nn ? A : a.nn - 1;
#pragma unroll
        for (int k = 0; k < ND; ++k) qv[A][k] = ld_q<T, ND>(a.q_in, b, a.nn, A, k, V, uv);
        sv[A] = smooth(a, b, Ac, v);
    }
    // compute phase: labels u = exp(ell), their forward differences, the
    // implicit-label gradients and the projected flow steps
    float gu[NLMAX][ND];
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        const float u0 = __expf(e0[L]);
#pragma unroll
        for (int k = 0; k < ND; ++k) gu[L][k] = h[k] ? __expf(en[L][k]) - u0 : 0.f;
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
                    flow_project<ND>(a, qv[A + j], G, h, sv[A + j], p[j]);
                }
            }
#pragma unroll
            for (int k = 0; k < ND; ++k) st_q2<T, ND>(a.q_out, b, a.nn, A, k, V, uv, p[0][k], p[1][k]);
        }
    }
}

template <int ND, int NLMAX, int NNMAX, bool IDENT, typename T>
__global__ __launch_bounds__(kBlock) void k_flow(StepArgs a) {
    flow_body<ND, NLMAX, NNMAX, IDENT, T>(a);
}

// --------------------------------------------- LDS-resident 2-D solve ----
// A 2-D problem whose float32 state fits in one compute unit's LDS (the
// 64 x 64 image with 3 labels: 147 KB) runs many iterations per launch: one
// block per problem loads ell and q into LDS, performs the label pass and
// the flow pass of every iteration there (a barrier after each), and stores
// the state back.  Each thread has up to kLdsVox voxels (the loops over them
// are unrolled, so their LDS reads overlap) and keeps their data terms in
// registers for the whole launch, so no global load waits inside the
// iterations but the capacities'.  LDS holds each value as the storage type
// holds it (every store goes through the same rounding) and each voxel's
// expressions are those of label_body / flow_body, so the result equals the
// two-pass kernels' bit for bit; at this size those are bound by launch
// latency (two launches per iteration, a few thousand voxels each).
template <int NLMAX, int NNMAX, bool IDENT, typename T>
__global__ __launch_bounds__(kLdsThreads) void k_lds2d(StepArgs a, int iters) {
    __shared__ float sm[kLdsFloats];
    const int b = blockIdx.x;
    const int V = a.V;
    const size_t Vs = (size_t)V;
    float *se = sm;                          // ell [nl][V]
    float *sq = sm + (size_t)a.nl * V;       // q [nn][2][V]
    const T *Tn = nullptr;
    float dr[kLdsVox][NLMAX];                // data terms of the thread's voxels
    int cx[kLdsVox], cy[kLdsVox];            // and their coordinates
#pragma unroll
    for (int j = 0; j < kLdsVox; ++j) {
        const int v = threadIdx.x + j * kLdsThreads;
        const unsigned vc = (unsigned)(v < V ? v : V - 1);
        cx[j] = (int)vc % a.nx;
        cy[j] = (int)vc / a.nx;
#pragma unroll
        for (int L = 0; L < NLMAX; ++L)
            dr[j][L] = ldf(field<float>(a.D, b, a.nl, L < a.nl ? L : a.nl - 1, Vs), vc);
        if (v < V) {
            for (int L = 0; L < a.nl; ++L) se[L * V + v] = ld_ell<T>(a.ell_in, b, a.nl, L, Vs, (unsigned)v);
            for (int A = 0; A < a.nn; ++A)
                for (int k = 0; k < 2; ++k)
                    sq[(A * 2 + k) * V + v] = ld_q<T, 2>(a.q_in, b, a.nn, A, k, Vs, (unsigned)v);
        }
    }
    __syncthreads();
    for (int it = 0; it < iters; ++it) {
        // label pass (label_body).  The voxel index is made opaque per
        // iteration so that the LDS addresses derived from it are formed
        // where they are used instead of being kept live across iterations.
#pragma unroll
        for (int j = 0; j < kLdsVox; ++j) {
            if (threadIdx.x + j * kLdsThreads < V) {
                int v = cy[j] * a.nx + cx[j];
                __asm__ volatile("" : "+v"(v));
                const Coord c{cx[j], cy[j], 0};
                int m[3];
                bool bwd[3];
                backward_offsets(c, a, m, bwd);
                const bool fwd[3] = {c.x < a.nx - 1, c.y < a.ny - 1, false};
                float d[NLMAX], e[NLMAX], q0[NNMAX][3], qm[NNMAX][3];
#pragma unroll
                for (int L = 0; L < NLMAX; ++L) {
                    d[L] = dr[j][L];
                    e[L] = se[(L < a.nl ? L : a.nl - 1) * V + v];
                }
#pragma unroll
                for (int A = 0; A < NNMAX; ++A) {
                    const int Ac = A < a.nn ? A : a.nn - 1;
#pragma unroll
                    for (int k = 0; k < 2; ++k) {
                        q0[A][k] = sq[(Ac * 2 + k) * V + v];
                        qm[A][k] = sq[(Ac * 2 + k) * V + v - m[k]];
                    }
                }
#pragma unroll
                for (int A = 0; A < NNMAX; ++A)
                    add_excess<NLMAX, IDENT>(a, d, A, div_from<2>(q0[A], qm[A], fwd, bwd));
                entropic_step<NLMAX>(a, d, e);
#pragma unroll
                for (int L = 0; L < NLMAX; ++L)
                    if (L < a.nl) se[L * V + v] = roundtrip(e[L], Tn);
            }
        }
        __syncthreads();
        // flow pass (flow_body)
#pragma unroll
        for (int j = 0; j < kLdsVox; ++j) {
            if (threadIdx.x + j * kLdsThreads < V) {
                int v = cy[j] * a.nx + cx[j];
                __asm__ volatile("" : "+v"(v));
                const Coord c{cx[j], cy[j], 0};
                const bool h[3] = {c.x < a.nx - 1, c.y < a.ny - 1, false};
                const int off[2] = {h[0] ? 1 : 0, h[1] ? a.nx : 0};
                float gu[NLMAX][2];
#pragma unroll
                for (int L = 0; L < NLMAX; ++L) {
                    const int Lc = L < a.nl ? L : a.nl - 1;
                    const float u0 = __expf(se[Lc * V + v]);
#pragma unroll
                    for (int k = 0; k < 2; ++k) gu[L][k] = h[k] ? __expf(se[Lc * V + v + off[k]]) - u0 : 0.f;
                }
#pragma unroll
                for (int A = 0; A < NNMAX; ++A) {
                    if (A < a.nn) {
                        const float qv[2] = {sq[(A * 2) * V + v], sq[(A * 2 + 1) * V + v]};
                        float G[3], p[2];
                        grad_U<2, NLMAX, IDENT>(a, A, gu, G);
                        flow_project<2>(a, qv, G, h, smooth(a, b, A, v), p);
                        sq[(A * 2) * V + v] = roundtrip(p[0], Tn);
                        sq[(A * 2 + 1) * V + v] = roundtrip(p[1], Tn);
                    }
                }
            }
        }
        __syncthreads();
    }
    for (int v = threadIdx.x; v < V; v += kLdsThreads) {
        for (int L = 0; L < a.nl; L += 2)
            st_ell2<T>(a.ell_out, b, a.nl, L, Vs, (unsigned)v, se[L * V + v],
                       L + 1 < a.nl ? se[(L + 1) * V + v] : 0.f);
        for (int A = 0; A < a.nn; A += 2)
            for (int k = 0; k < 2; ++k)
                st_q2<T, 2>(a.q_out, b, a.nn, A, k, Vs, (unsigned)v, sq[(A * 2 + k) * V + v],
                            A + 1 < a.nn ? sq[((A + 1) * 2 + k) * V + v] : 0.f);
    }
}

// the builds of the LDS-resident solve (up to 8 leaves and 16 flows)
template <typename T, typename F>
hipError_t lds_bucket(bool ident, int nl, int nn, F &f) {
    if (ident) {
        if (nl <= 4) return f.template operator()<4, 4, true, T>();
        return f.template operator()<8, 8, true, T>();
    }
    if (nl <= 4 && nn <= 8) return f.template operator()<4, 8, false, T>();
    if (nl <= 8 && nn <= 8) return f.template operator()<8, 8, false, T>();
    if (nl <= 8 && nn <= 12) return f.template operator()<8, 12, false, T>();
    return f.template operator()<8, 16, false, T>();
}

// ------------------------------- LDS tiles with ghost zones (2-D) -------
// A problem too small to fill the GPU (one 64 x 64 image) is bound by launch
// latency in the two-pass kernels (two launches per iteration) and by one
// compute unit's issue rate when it sits in one block (k_lds2d).  Here each
// block owns a tile of g.ox x g.oy voxels and loads the tile plus a ghost
// zone g.k voxels wide on each side (clipped at the image border) into LDS,
// then performs up to g.k iterations there and stores its own tile.  The
// label step at x reads flows at x - e_k and the flow step reads labels at
// x + e_k, so each iteration leaves one more ghost layer stale on each side
// and the owned tile is exact after g.k of them; the stale ghost values are
// never read by an owned voxel, and reads past the loaded region are
// clamped into it.  Blocks read the previous launch's state and write the
// other buffer, so no launch reads what one of its blocks writes.  One voxel
// per thread, the thread's data terms and capacities in registers, fields in
// LDS at a stride of one float per thread; each voxel evaluates k_lds2d's
// expressions (those of label_body / flow_body) with the same roundings, so
// the result equals the two-pass kernels' bit for bit.
template <int NLMAX, int NNMAX, bool IDENT, typename T>
__global__ __launch_bounds__(tile_threads(NNMAX)) void k_tile2d(StepArgs a, TileGeom g, int iters) {
    constexpr int R = tile_threads(NNMAX);
    __shared__ float se[NLMAX * R];            // ell [nl][R]
    __shared__ float sq[NNMAX * 2 * R];        // q [nn][2][R]
    const T *Tn = nullptr;
    const int tiles = g.tiles_x * g.tiles_y;
    const int b = blockIdx.x / tiles;
    const int tl = blockIdx.x - b * tiles;
    const int ox0 = (tl % g.tiles_x) * g.ox, oy0 = (tl / g.tiles_x) * g.oy;
    const int rx0 = max(0, ox0 - g.k), ry0 = max(0, oy0 - g.k);
    const int rw = min(a.nx, ox0 + g.ox + g.k) - rx0;     // this block's region
    const int rh = min(a.ny, oy0 + g.oy + g.k) - ry0;
    const int lx = (int)threadIdx.x % g.rw, ly = (int)threadIdx.x / g.rw;
    const bool act = ly < g.rh && lx < rw && ly < rh;
    const int x = rx0 + (act ? lx : 0), y = ry0 + (act ? ly : 0);
    const int r = ly * g.rw + lx;
    const size_t Vs = (size_t)a.V;
    const unsigned v = (unsigned)(y * a.nx + x);
    // LDS neighbours, clamped into the region
    const int rxm = lx > 0 ? r - 1 : r, rym = ly > 0 ? r - g.rw : r;
    const int rxp = lx < rw - 1 ? r + 1 : r, ryp = ly < rh - 1 ? r + g.rw : r;
    const bool bwd[3] = {x > 0, y > 0, false};
    const bool fwd[3] = {x < a.nx - 1, y < a.ny - 1, false};
    float dr[NLMAX], sv[NNMAX];
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) dr[L] = ldf(field<float>(a.D, b, a.nl, L < a.nl ? L : a.nl - 1, Vs), v);
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) sv[A] = smooth(a, b, A < a.nn ? A : a.nn - 1, (int)v);
    if (act) {
#pragma unroll
        for (int L = 0; L < NLMAX; ++L)
            if (L < a.nl) se[L * R + r] = ld_ell<T>(a.ell_in, b, a.nl, L, Vs, v);
#pragma unroll
        for (int A = 0; A < NNMAX; ++A)
            if (A < a.nn)
#pragma unroll
                for (int k = 0; k < 2; ++k) sq[(A * 2 + k) * R + r] = ld_q<T, 2>(a.q_in, b, a.nn, A, k, Vs, v);
    }
    __syncthreads();
    for (int it = 0; it < iters; ++it) {
        if (act) {
            // label step (label_body)
            float d[NLMAX], e[NLMAX], q0[NNMAX][3], qm[NNMAX][3];
#pragma unroll
            for (int L = 0; L < NLMAX; ++L) {
                d[L] = dr[L];
                e[L] = se[(L < a.nl ? L : a.nl - 1) * R + r];
            }
#pragma unroll
            for (int A = 0; A < NNMAX; ++A) {
                const int Ac = A < a.nn ? A : a.nn - 1;
                q0[A][0] = sq[(Ac * 2) * R + r];
                q0[A][1] = sq[(Ac * 2 + 1) * R + r];
                qm[A][0] = sq[(Ac * 2) * R + rxm];
                qm[A][1] = sq[(Ac * 2 + 1) * R + rym];
            }
#pragma unroll
            for (int A = 0; A < NNMAX; ++A)
                add_excess<NLMAX, IDENT>(a, d, A, div_from<2>(q0[A], qm[A], fwd, bwd));
            entropic_step<NLMAX>(a, d, e);
#pragma unroll
            for (int L = 0; L < NLMAX; ++L)
                if (L < a.nl) se[L * R + r] = roundtrip(e[L], Tn);
        }
        __syncthreads();
        if (act) {
            // flow step (flow_body)
            const bool h[3] = {fwd[0], fwd[1], false};
            const int nb[2] = {rxp, ryp};
            float gu[NLMAX][2];
#pragma unroll
            for (int L = 0; L < NLMAX; ++L) {
                const int Lc = L < a.nl ? L : a.nl - 1;
                const float u0 = __expf(se[Lc * R + r]);
#pragma unroll
                for (int k = 0; k < 2; ++k) gu[L][k] = h[k] ? __expf(se[Lc * R + nb[k]]) - u0 : 0.f;
            }
#pragma unroll
            for (int A = 0; A < NNMAX; ++A) {
                if (A < a.nn) {
                    const float qv[2] = {sq[(A * 2) * R + r], sq[(A * 2 + 1) * R + r]};
                    float G[3], p[2];
                    grad_U<2, NLMAX, IDENT>(a, A, gu, G);
                    flow_project<2>(a, qv, G, h, sv[A], p);
                    sq[(A * 2) * R + r] = roundtrip(p[0], Tn);
                    sq[(A * 2 + 1) * R + r] = roundtrip(p[1], Tn);
                }
            }
        }
        __syncthreads();
    }
    // store the owned tile
    if (act && x >= ox0 && x < ox0 + g.ox && y >= oy0 && y < oy0 + g.oy) {
#pragma unroll
        for (int L = 0; L < NLMAX; L += 2)
            if (L < a.nl)
                st_ell2<T>(a.ell_out, b, a.nl, L, Vs, v, se[L * R + r],
                           L + 1 < a.nl ? se[(L + 1) * R + r] : 0.f);
#pragma unroll
        for (int A = 0; A < NNMAX; A += 2)
            if (A < a.nn)
#pragma unroll
                for (int k = 0; k < 2; ++k)
                    st_q2<T, 2>(a.q_out, b, a.nn, A, k, Vs, v, sq[(A * 2 + k) * R + r],
                                A + 1 < a.nn ? sq[((A + 1) * 2 + k) * R + r] : 0.f);
    }
}

// ------------------------------------------------- init / copy / export --

template <typename T>
__global__ __launch_bounds__(kBlock) void k_init(T *ell, size_t n_ell, T *q, size_t n_q,
                                                 float ell0) {
    const size_t stride = (size_t)gridDim.x * kBlock;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n_ell; i += stride)
        st(ell, i, ell0);
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n_q; i += stride)
        st(q, i, 0.f);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(const T *__restrict__ a, T *__restrict__ b,
                                                 size_t n, const T *__restrict__ c,
                                                 T *__restrict__ d, size_t m) {
    const size_t stride = (size_t)gridDim.x * kBlock;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) b[i] = a[i];
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) d[i] = c[i];
}

template <int ND, typename T>
__global__ __launch_bounds__(kBlock) void k_export(StepArgs a, float *u, int32_t *labels,
                                                   float *qo) {
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= a.V) return;
    const int b = blockIdx.y;
    const size_t V = (size_t)a.V;
    int best = 0;
    float bv = -INFINITY;
    for (int L = 0; L < a.nl; ++L) {
        const size_t i = ((size_t)b * a.nl + L) * V + v;
        const float e = ld_ell<T>(a.ell_in, b, a.nl, L, V, (unsigned)v);
        if (u) u[i] = expf(e);
        if (e > bv) {
            bv = e;
            best = L;
        }
    }
    if (labels) labels[(size_t)b * V + v] = best;
    if (qo) {
        for (int A = 0; A < a.nn; ++A)
            for (int k = 0; k < ND; ++k)
                qo[((size_t)b * a.nn * ND + A * ND + k) * V + v] =
                    ld_q<T, ND>(a.q_in, b, a.nn, A, k, V, (unsigned)v);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_export_ell(StepArgs a, float *out) {
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= a.V) return;
    const int b = blockIdx.y;
    const size_t V = (size_t)a.V;
    for (int L = 0; L < a.nl; ++L)
        out[((size_t)b * a.nl + L) * V + v] = ld_ell<T>(a.ell_in, b, a.nl, L, V, (unsigned)v);
}

__global__ __launch_bounds__(kBlock) void k_check(const float *D, size_t nD, const float *S,
                                                  size_t nS, int32_t *flag) {
    const size_t stride = (size_t)gridDim.x * kBlock;
    int bad = 0;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < nD; i += stride)
        bad |= !isfinite(D[i]);
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < nS; i += stride)
        bad |= !(isfinite(S[i]) && S[i] >= 0.f) ? 2 : 0;
    if (bad) atomicOr(flag, bad);
}

__global__ __launch_bounds__(kBlock) void k_upload(ConstBlock c, float *dst) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < PF_MAX_NODES) dst[i] = c.s_node[i];
    else if (i < kConstFloats) dst[i] = c.w[i - PF_MAX_NODES];
}

__global__ void k_zero_flag(int32_t *flag) {
    if (threadIdx.x == 0) flag[0] = 0;
}

// ---------------------------------------------------- energy and dual ----

// Per block: sum of E, sum of P, max |sum u - 1|, max(|q_A| - S_A), in fp64.
template <int ND, int NLMAX, int NNMAX, bool IDENT, typename T>
__device__ __forceinline__ void energy_body(const StepArgs &a, double *partials) {
    __shared__ double red[4][kBlock];
    // path weights staged in LDS once per block: read in the voxel loop
    // without scalar-memory waits (they are 0 outside the graph)
    __shared__ float wsh[IDENT ? 1 : NNMAX * NLMAX];
    if constexpr (!IDENT) {
        for (int i = threadIdx.x; i < NNMAX * NLMAX; i += kBlock)
            wsh[i] = wgt(a, i / NLMAX, i % NLMAX);
        __syncthreads();
    }
    const size_t V = (size_t)a.V;
    const size_t total = V * a.B;
    double e_sum = 0.0, p_sum = 0.0, mx_s = 0.0, mx_q = -INFINITY;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        // compiler-only memory barrier (no instruction): keeps the LDS weight
        // reads inside the loop instead of hoisting all of them into registers
        asm volatile("" ::: "memory");
        const int b = (int)(i / V);
        const int v = (int)(i - (size_t)b * V);
        const Coord c = coord_of(v, a.nx, a.ny);
        const bool h[3] = {c.x < a.nx - 1, c.y < a.ny - 1, ND == 3 && c.z < a.nz - 1};
        const int off[3] = {h[0] ? 1 : 0, h[1] ? a.nx : 0, h[2] ? a.nx * a.ny : 0};
        int m[3];
        bool bwd[3];
        backward_offsets(c, a, m, bwd);
        const unsigned uv = (unsigned)v;
        // load phase (unconditional, clamped indices), as in the iteration kernels
        float e0[NLMAX], en[NLMAX][ND], dl[NLMAX], q0[NNMAX][3], qm[NNMAX][3], sv[NNMAX];
#pragma unroll
        for (int L = 0; L < NLMAX; ++L) {
            e0[L] = ld_ell<T>(a.ell_in, b, a.nl, L, V, uv);
#pragma unroll
            for (int k = 0; k < ND; ++k) en[L][k] = ld_ell<T>(a.ell_in, b, a.nl, L, V, uv + (unsigned)off[k]);
            dl[L] = ldf(field<float>(a.D, b, a.nl, L < a.nl ? L : a.nl - 1, V), uv);
        }
#pragma unroll
        for (int A = 0; A < NNMAX; ++A) {
#pragma unroll
            for (int k = 0; k < 3; ++k) q0[A][k] = qm[A][k] = 0.f;
#pragma unroll
            for (int k = 0; k < ND; ++k) {
                q0[A][k] = ld_q<T, ND>(a.q_in, b, a.nn, A, k, V, uv);
                qm[A][k] = ld_q<T, ND>(a.q_in, b, a.nn, A, k, V, uv - (unsigned)m[k]);
            }
            sv[A] = smooth(a, b, A < a.nn ? A : a.nn - 1, v);
        }
        // labels at x and at the forward neighbours (float32 exp of the stored
        // state), every product and sum in float64
        float u[NLMAX], un[NLMAX][ND];
        double d[NLMAX];
        double su = 0.0, e = 0.0;
#pragma unroll
        for (int L = 0; L < NLMAX; ++L) {
            u[L] = expf(e0[L]);
#pragma unroll
            for (int k = 0; k < ND; ++k) un[L][k] = h[k] ? expf(en[L][k]) : u[L];
            d[L] = (double)dl[L];
            if (L < a.nl) {
                su += (double)u[L];
                e += d[L] * (double)u[L];
            }
        }
#pragma unroll
        for (int A = 0; A < NNMAX; ++A) {
            if (A < a.nn) {
                double G[ND];
#pragma unroll
                for (int k = 0; k < ND; ++k) G[k] = 0.0;
                if constexpr (IDENT) {
#pragma unroll
                    for (int k = 0; k < ND; ++k) G[k] = (double)un[A][k] - (double)u[A];
                } else {
#pragma unroll
                    for (int L = 0; L < NLMAX; ++L) {
                        const double wl = (double)wsh[A * NLMAX + L];
#pragma unroll
                        for (int k = 0; k < ND; ++k) G[k] += wl * ((double)un[L][k] - (double)u[L]);
                    }
                }
                double n2 = 0.0;
#pragma unroll
                for (int k = 0; k < ND; ++k) n2 += G[k] * G[k];
                const double S = (double)sv[A];
                e += S * sqrt(n2);
                // flow excess over the capacity and divergence, fp64
                double qn2 = 0.0, dv = 0.0;
#pragma unroll
                for (int k = 0; k < ND; ++k) {
                    const double qk = q0[A][k];
                    qn2 += qk * qk;
                    dv += h[k] ? qk : 0.0;
                    dv -= bwd[k] ? (double)qm[A][k] : 0.0;
                }
                mx_q = fmax(mx_q, sqrt(qn2) - S);
                if constexpr (IDENT) {
                    d[A] += dv;
                } else {
#pragma unroll
                    for (int L = 0; L < NLMAX; ++L) d[L] += (double)wsh[A * NLMAX + L] * dv;
                }
            }
        }
        double pm = INFINITY;
#pragma unroll
        for (int L = 0; L < NLMAX; ++L)
            if (L < a.nl) pm = fmin(pm, d[L]);
        e_sum += e;
        p_sum += pm;
        mx_s = fmax(mx_s, fabs(su - 1.0));
    }
    red[0][threadIdx.x] = e_sum;
    red[1][threadIdx.x] = p_sum;
    red[2][threadIdx.x] = mx_s;
    red[3][threadIdx.x] = mx_q;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
            red[2][threadIdx.x] = fmax(red[2][threadIdx.x], red[2][threadIdx.x + s]);
            red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) partials[blockIdx.x * 4 + j] = red[j][0];
    }
}

template <int ND, int NLMAX, int NNMAX, bool IDENT, typename T>
__global__ __launch_bounds__(kBlock) void k_energy(StepArgs a, double *partials) {
    energy_body<ND, NLMAX, NNMAX, IDENT, T>(a, partials);
}

// Fixed-order final reduction of the block partials (deterministic).
__global__ __launch_bounds__(kBlock) void k_reduce(const double *partials, int n,
                                                   double *results) {
    __shared__ double red[4][kBlock];
    double s0 = 0.0, s1 = 0.0, m2 = 0.0, m3 = -INFINITY;
    for (int i = threadIdx.x; i < n; i += kBlock) {
        s0 += partials[i * 4 + 0];
        s1 += partials[i * 4 + 1];
        m2 = fmax(m2, partials[i * 4 + 2]);
        m3 = fmax(m3, partials[i * 4 + 3]);
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    red[2][threadIdx.x] = m2;
    red[3][threadIdx.x] = m3;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
            red[2][threadIdx.x] = fmax(red[2][threadIdx.x], red[2][threadIdx.x + s]);
            red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        results[0] = red[0][0];
        results[1] = red[1][0];
        results[2] = red[2][0];
        results[3] = red[3][0];
    }
}

// ----------------------------------------------------------- dispatch ----

template <int ND, typename T, typename F>
hipError_t by_bucket(bool ident, int nl, int nn, F &f) {
    if (ident) {
        if (nl <= 4) return f.template operator()<ND, 4, 4, true, T>();
        if (nl <= 8) return f.template operator()<ND, 8, 8, true, T>();
        return f.template operator()<ND, 16, 16, true, T>();
    }
    if (nl <= 4 && nn <= 8) return f.template operator()<ND, 4, 8, false, T>();
    if (nl <= 8 && nn <= 8) return f.template operator()<ND, 8, 8, false, T>();
    if (nl <= 8 && nn <= 12) return f.template operator()<ND, 8, 12, false, T>();
    if (nl <= 8 && nn <= 16) return f.template operator()<ND, 8, 16, false, T>();
    if (nl <= 12 && nn <= 16) return f.template operator()<ND, 12, 16, false, T>();
    if (nn <= 16) return f.template operator()<ND, 16, 16, false, T>();
    return f.template operator()<ND, 16, 32, false, T>();
}

template <typename F>
hipError_t dispatch(int nd, int storage, bool ident, int nl, int nn, F &&f) {
    if (nd == 2) {
        if (storage == PF_BF16) return by_bucket<2, bf16s>(ident, nl, nn, f);
        if (storage == PF_FP16) return by_bucket<2, f16s>(ident, nl, nn, f);
        return by_bucket<2, float>(ident, nl, nn, f);
    }
    if (storage == PF_BF16) return by_bucket<3, bf16s>(ident, nl, nn, f);
    if (storage == PF_FP16) return by_bucket<3, f16s>(ident, nl, nn, f);
    return by_bucket<3, float>(ident, nl, nn, f);
}

template <typename F>
hipError_t dispatch_type(int storage, F &&f) {
    if (storage == PF_BF16) return f.template operator()<bf16s>();
    if (storage == PF_FP16) return f.template operator()<f16s>();
    return f.template operator()<float>();
}

dim3 voxel_grid(const StepArgs &a) {
    return dim3((unsigned)((a.V + kBlock - 1) / kBlock), (unsigned)a.B, 1);
}

unsigned stride_blocks(size_t n) {
    const size_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < 4096 ? (b ? b : 1) : 4096);
}

}  // namespace

// ---------------------------------------------------------- launchers ----

size_t storage_bytes(int storage) { return storage == PF_FP32 ? 4 : 2; }

hipError_t launch_init(const StepArgs &a, int nd, int storage, float ell0, hipStream_t s) {
    const size_t n_ell = (size_t)a.B * state_fields(a.nl, storage) * a.V;
    const size_t n_q = (size_t)a.B * state_fields(a.nn, storage) * nd * a.V;
    return dispatch_type(storage, [&]<typename T>() {
        k_init<T><<<stride_blocks(n_ell > n_q ? n_ell : n_q), kBlock, 0, s>>>(
            static_cast<T *>(a.ell_out), n_ell, static_cast<T *>(a.q_out), n_q, ell0);
        return hipGetLastError();
    });
}

hipError_t launch_copy_state(const StepArgs &a, int nd, int storage, hipStream_t s) {
    const size_t n_ell = (size_t)a.B * state_fields(a.nl, storage) * a.V;
    const size_t n_q = (size_t)a.B * state_fields(a.nn, storage) * nd * a.V;
    return dispatch_type(storage, [&]<typename T>() {
        k_copy<T><<<stride_blocks(n_q), kBlock, 0, s>>>(
            static_cast<const T *>(a.ell_in), static_cast<T *>(a.ell_out), n_ell,
            static_cast<const T *>(a.q_in), static_cast<T *>(a.q_out), n_q);
        return hipGetLastError();
    });
}

hipError_t launch_upload(const ConstBlock &c, float *dst, hipStream_t s) {
    k_upload<<<(kConstFloats + kBlock - 1) / kBlock, kBlock, 0, s>>>(c, dst);
    return hipGetLastError();
}

bool lds_supported(int nd, int nl, int nn, long V) {
    return nd == 2 && nl <= 8 && nn <= 16 && V > 0 && V <= (long)kLdsVox * kLdsThreads &&
           V * (long)(nl + 2 * nn) <= kLdsFloats;
}

// PF_KERNEL_AUTO takes the LDS-resident solve from 8 problems up: one compute
// unit per problem and no HBM traffic per iteration (64 x 64, 3 labels, 200
// iterations: batch 256 1.55 against 4.5 ms for the two-pass kernels, batch
// 8 1.53 against 1.59 ms); a single problem runs on one compute unit and is
// no faster than the two-pass kernels' launches (1.52 against 1.49 ms).
bool lds_preferred(int nd, int nl, int nn, long V, int batch) {
    return batch >= 8 && lds_supported(nd, nl, nn, V);
}

hipError_t launch_lds(const StepArgs &a, bool ident, int storage, int iters, hipStream_t s) {
    if (!lds_supported(2, a.nl, a.nn, a.V) || a.nz != 1 || iters < 1) return hipErrorInvalidValue;
    return dispatch_type(storage, [&]<typename T>() {
        auto go = [&]<int NL, int NN, bool ID, typename U>() {
            k_lds2d<NL, NN, ID, U><<<(unsigned)a.B, kLdsThreads, 0, s>>>(a, iters);
            return hipGetLastError();
        };
        return lds_bucket<T>(ident, a.nl, a.nn, go);
    });
}

bool tile_supported(int nd, int nl, int nn) { return nd == 2 && nl <= 8 && nn <= 16; }

// Owned tiles of 16 x 16 voxels with ghost zones 8 wide (8 iterations per
// launch, a region of up to 32 x 32 voxels per block) while the problems give
// at least 64 tiles and the build has at most 8 flows; otherwise 8 x 8 owned
// (regions of up to 24 x 24).
TileGeom tile_geometry(int nx, int ny, int batch, int nn) {
    TileGeom g{};
    g.k = 8;
    g.ox = g.oy = 16;
    if (nn > 8 || (long)((nx + 15) / 16) * ((ny + 15) / 16) * batch < 64) g.ox = g.oy = 8;
    g.rw = nx < g.ox + 2 * g.k ? nx : g.ox + 2 * g.k;
    g.rh = ny < g.oy + 2 * g.k ? ny : g.oy + 2 * g.k;
    g.tiles_x = (nx + g.ox - 1) / g.ox;
    g.tiles_y = (ny + g.oy - 1) / g.oy;
    return g;
}

// PF_KERNEL_AUTO takes the tiles for 2-D problems of at most 8 flows that
// the whole-problem LDS solve does not take, up to 2^21 voxel-fields
// (voxels x problems x (n_leaf + n_node)), where they measured faster than
// the two-pass kernels on MI355X (per solve: 64 x 64 with 3 labels, 200
// iterations, 0.49 against 1.26 ms, and 7 such problems 0.56 against 1.27;
// 512 x 512 with 3 labels, 50 iterations, 0.40 against 0.69 ms; beyond:
// 1024 x 1024 with 3 labels 1.25 against 1.34 ms, a 512 x 512 DAG of 5
// leaves and 8 flows 1.23 against 0.95 ms).  The builds of more than 8
// flows have 24 x 24 regions (9x the owned voxels) and stay with two-pass.
bool tile_preferred(int nd, int nl, int nn, long V, int batch) {
    return tile_supported(nd, nl, nn) && nn <= 8 && !lds_preferred(nd, nl, nn, V, batch) &&
           V * batch * (nl + nn) <= (1L << 21);
}

hipError_t launch_tile(const StepArgs &a, bool ident, int storage, int iters, hipStream_t s) {
    if (!tile_supported(2, a.nl, a.nn) || a.nz != 1 || iters < 1) return hipErrorInvalidValue;
    const TileGeom g = tile_geometry(a.nx, a.ny, a.B, a.nn);
    const long blocks = (long)g.tiles_x * g.tiles_y * a.B;
    if (iters > g.k || blocks <= 0 || blocks > 0x7fffffffL) return hipErrorInvalidValue;
    return dispatch_type(storage, [&]<typename T>() {
        auto go = [&]<int NL, int NN, bool ID, typename U>() {
            if (g.rw * g.rh > tile_threads(NN)) return hipErrorInvalidValue;
            k_tile2d<NL, NN, ID, U><<<(unsigned)blocks, tile_threads(NN), 0, s>>>(a, g, iters);
            return hipGetLastError();
        };
        return lds_bucket<T>(ident, a.nl, a.nn, go);
    });
}

hipError_t launch_label(const StepArgs &a, bool ident, int nd, int storage, hipStream_t s) {
    return dispatch(nd, storage, ident, a.nl, a.nn,
                    [&]<int ND, int NL, int NN, bool ID, typename T>() {
                        k_label<ND, NL, NN, ID, T><<<voxel_grid(a), kBlock, 0, s>>>(a);
                        return hipGetLastError();
                    });
}

hipError_t launch_flow(const StepArgs &a, bool ident, int nd, int storage, hipStream_t s) {
    return dispatch(nd, storage, ident, a.nl, a.nn,
                    [&]<int ND, int NL, int NN, bool ID, typename T>() {
                        k_flow<ND, NL, NN, ID, T><<<voxel_grid(a), kBlock, 0, s>>>(a);
                        return hipGetLastError();
                    });
}

hipError_t launch_energy(const StepArgs &a, bool ident, int nd, int storage,
                         double *partials, double *results, hipStream_t s) {
    hipError_t e = dispatch(nd, storage, ident, a.nl, a.nn,
                            [&]<int ND, int NL, int NN, bool ID, typename T>() {
                                k_energy<ND, NL, NN, ID, T>
                                    <<<kPartials, kBlock, 0, s>>>(a, partials);
                                return hipGetLastError();
                            });
    if (e != hipSuccess) return e;
    k_reduce<<<1, kBlock, 0, s>>>(partials, kPartials, results);
    return hipGetLastError();
}

hipError_t launch_export(const StepArgs &a, int nd, int storage, float *u, int32_t *labels,
                         float *q, hipStream_t s) {
    return dispatch_type(storage, [&]<typename T>() {
        if (nd == 2)
            k_export<2, T><<<voxel_grid(a), kBlock, 0, s>>>(a, u, labels, q);
        else
            k_export<3, T><<<voxel_grid(a), kBlock, 0, s>>>(a, u, labels, q);
        return hipGetLastError();
    });
}

hipError_t launch_export_ell(const StepArgs &a, int storage, float *ell, hipStream_t s) {
    return dispatch_type(storage, [&]<typename T>() {
        k_export_ell<T><<<voxel_grid(a), kBlock, 0, s>>>(a, ell);
        return hipGetLastError();
    });
}

hipError_t launch_check(const StepArgs &a, int32_t *flag, hipStream_t s) {
    k_zero_flag<<<1, 64, 0, s>>>(flag);
    const size_t nD = (size_t)a.B * a.nl * a.V;
    size_t nS = 0;
    if (a.s_mode == PF_S_SHARED_FIELD) nS = (size_t)a.B * a.V;
    if (a.s_mode == PF_S_NODE_FIELD) nS = (size_t)a.B * a.nn * a.V;
    k_check<<<stride_blocks(nD), kBlock, 0, s>>>(a.D, nD, a.S, nS, flag);
    return hipGetLastError();
}

}  // namespace pf
