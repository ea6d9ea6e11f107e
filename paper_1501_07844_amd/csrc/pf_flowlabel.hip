// Single pass per iteration for label graphs (DAGMF, HMF and the Ishikawa
// chain) on 3-D grids: the flow step of iteration k followed, at the same
// voxel, by the label step of iteration k + 1.
//
// The label-then-flow fused pass (pf_fused.hip) needs, for the flow step at
// plane z, the new labels of plane z + 1, so it holds the old flows of two
// planes in registers: 96 values for 16 flows, which spills.  Shifting the
// pass boundary by half an iteration reverses the dependency.  The flow step
// of iteration k at x reads the labels after label step k at x and x + e_k,
// which the previous pass wrote (read-only here), and the old flows at x; the
// label step of iteration k + 1 at x then needs the new flows at x and at the
// backward neighbours x - e_k:
//   z - 1: the thread's own previous plane (its rounded q_z, in registers);
//   x - 1, y - 1: neighbouring threads of the plane, through LDS; the column
//          x0 - 1 and the row y0 - 1 of a tile belong to neighbouring tiles,
//          and halo threads recompute their flow steps (no label step).
// Only one plane of flows is live per thread, and the z neighbour of a flow
// step is a plain load, so a chunk of planes needs one extra flow step (the
// plane below the chunk, for its q_z) and nothing past its end.
//
// The state between passes is (labels of iteration k + 1, flows of
// iteration k).  A solve enters it with one label pass and leaves it with one
// flow pass (the two-pass kernels, in place), around every gap check and at
// the end; n iterations between two checks cost n - 1 of these passes plus
// the two half passes.
//
// Each voxel evaluates the expressions of the two-pass kernels in their order
// (the flow step of flow_body, the label step of label_body), with the new
// flows rounded to the storage type where the two-pass label pass would load
// them, so the result equals the two-pass kernels' bit for bit.

#include <hip/hip_runtime.h>
#include <math.h>

#include "pf_device.h"
#include "pf_internal.h"

namespace pf {
namespace {

using namespace dev;

constexpr int GX = 64;                     // tile width (one wavefront per row)
constexpr int GY = 8;                      // owned tile rows
constexpr int GTHREADS = GX * (GY + 2);    // owned rows, the halo row, the halo column

// Flow step of iteration k at voxel (x, y, z): the labels of iteration k at
// the voxel (returned in e0, as stored) and at x + e_k, the old flows at the
// voxel and the capacities; returns the new flows after a round trip
// through the storage type (what a later load returns; 0 past the last
// flow) and stores them when `store`.
template <int NLMAX, int NNMAX, typename T>
__device__ __forceinline__ void flow_point(const StepArgs &a, int b, int x, int y, int z, bool store,
                                           float (&e0)[NLMAX], float (&pr)[NNMAX][3]) {
    const size_t V = (size_t)a.V;
    const unsigned uv = (unsigned)((z * a.ny + y) * a.nx + x);
    const bool h[3] = {x < a.nx - 1, y < a.ny - 1, z < a.nz - 1};
    const unsigned off[3] = {h[0] ? 1u : 0u, h[1] ? (unsigned)a.nx : 0u,
                             h[2] ? (unsigned)(a.nx * a.ny) : 0u};
    float en[NLMAX][3], qv[NNMAX][3], sv[NNMAX];
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        e0[L] = ld_ell<T>(a.ell_in, b, a.nl, L, V, uv);
#pragma unroll
        for (int k = 0; k < 3; ++k) en[L][k] = ld_ell<T>(a.ell_in, b, a.nl, L, V, uv + off[k]);
    }
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) {
#pragma unroll
        for (int k = 0; k < 3; ++k) qv[A][k] = ld_q<T, 3>(a.q_in, b, a.nn, A, k, V, uv);
        sv[A] = smooth(a, b, A < a.nn ? A : a.nn - 1, (int)uv);
    }
    float gu[NLMAX][3];
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        const float u0 = __expf(e0[L]);
#pragma unroll
        for (int k = 0; k < 3; ++k) gu[L][k] = h[k] ? __expf(en[L][k]) - u0 : 0.f;
    }
#pragma unroll
    for (int A = 0; A < NNMAX; A += 2) {
        float p[2][3];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            p[j][0] = p[j][1] = p[j][2] = 0.f;
            if (A + j < a.nn) {
                float G[3];
                grad_U<3, NLMAX, false>(a, A + j, gu, G);
                flow_project<3>(a, qv[A + j], G, h, sv[A + j], p[j]);
            }
        }
        if (store && A < a.nn) {
#pragma unroll
            for (int k = 0; k < 3; ++k) st_q2<T, 3>(a.q_out, b, a.nn, A, k, V, uv, p[0][k], p[1][k]);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) pr[A + j][k] = roundtrip(p[j][k], static_cast<const T *>(nullptr));
    }
}

template <int NLMAX, int NNMAX, typename T>
__global__ __launch_bounds__(GTHREADS) void k_flow_label(StepArgs a, FusedGeom g) {
    // new flows' x and y components: [flow][component][row + 1][column + 1],
    // row 0 the halo row y0 - 1 and column 0 the halo column x0 - 1
    __shared__ float lq[NNMAX][2][GY + 1][GX + 1];
    const int row = threadIdx.x / GX;      // GY: halo row, GY + 1: halo column
    const int col = threadIdx.x % GX;

    // XCD-aware block -> tile mapping (as in the fused kernels)
    const int nb = gridDim.x;
    const int pb = blockIdx.x;
    const int lb = (nb % 8 == 0) ? (pb % 8) * (nb / 8) + pb / 8 : pb;
    const int bx = lb % g.tiles_x;
    int r = lb / g.tiles_x;
    const int by = r % g.tiles_y;
    r /= g.tiles_y;
    const int ch = r % g.n_chunks;
    const int b = r / g.n_chunks;
    const int x0 = bx * GX, y0 = by * GY;
    const int zs = ch * g.cz;
    const int ze = min(a.nz, zs + g.cz);

    const bool colp = row == GY + 1;
    const int xa = colp ? x0 - 1 : x0 + col;
    const int ya = colp ? y0 + col : (row == GY ? y0 - 1 : y0 + row);
    const bool va = (!colp || col < GY) && xa >= 0 && ya >= 0 && xa < a.nx && ya < a.ny;
    const bool own = row < GY && va;
    const int lr = colp ? col + 1 : (row == GY ? 0 : row + 1);
    const int lc = colp ? 0 : col + 1;
    const size_t V = (size_t)a.V;

    // rounded q_z of the new flows one plane below (the z neighbour of the
    // divergence); a chunk that starts above plane 0 recomputes that plane
    float pzb[NNMAX];
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) pzb[A] = 0.f;
    if (own && zs > 0) {
        float e0[NLMAX], pr[NNMAX][3];
        flow_point<NLMAX, NNMAX, T>(a, b, xa, ya, zs - 1, false, e0, pr);
#pragma unroll
        for (int A = 0; A < NNMAX; ++A) pzb[A] = pr[A][2];
    }

    for (int z = zs; z < ze; ++z) {
        float e0[NLMAX], pz[NNMAX], dl[NLMAX];
        if (va) {
            float pr[NNMAX][3];
            flow_point<NLMAX, NNMAX, T>(a, b, xa, ya, z, own, e0, pr);
#pragma unroll
            for (int A = 0; A < NNMAX; ++A) {
                lq[A][0][lr][lc] = pr[A][0];
                lq[A][1][lr][lc] = pr[A][1];
                pz[A] = pr[A][2];
            }
        }
        if (own) {
            const unsigned uv = (unsigned)((z * a.ny + ya) * a.nx + xa);
#pragma unroll
            for (int L = 0; L < NLMAX; ++L)
                dl[L] = ldf(field<float>(a.D, b, a.nl, L < a.nl ? L : a.nl - 1, V), uv);
        }
        __syncthreads();
        // label step of iteration k + 1 (label_body's expressions and order)
        if (own) {
            const unsigned uv = (unsigned)((z * a.ny + ya) * a.nx + xa);
            const bool bwd[3] = {xa > 0, ya > 0, z > 0};
            const bool fwd[3] = {xa < a.nx - 1, ya < a.ny - 1, z < a.nz - 1};
#pragma unroll
            for (int A = 0; A < NNMAX; ++A) {
                const float q0[3] = {lq[A][0][lr][lc], lq[A][1][lr][lc], pz[A]};
                const float qm[3] = {lq[A][0][lr][lc - 1], lq[A][1][lr - 1][lc], pzb[A]};
                add_excess<NLMAX, false>(a, dl, A, div_from<3>(q0, qm, fwd, bwd));
            }
            entropic_step<NLMAX>(a, dl, e0);
#pragma unroll
            for (int L = 0; L < NLMAX; L += 2) st_ell2<T>(a.ell_out, b, a.nl, L, V, uv, e0[L], e0[L + 1]);
#pragma unroll
            for (int A = 0; A < NNMAX; ++A) pzb[A] = pz[A];
        }
        __syncthreads();   // the plane's LDS flows are read
    }
}

// ----------------------------------------------------------- dispatch ----

}  // namespace

bool flow_label_supported(int nd, int nl, int nn, bool identity) {
    return nd == 3 && !identity && nl <= 16 && nn <= 16;
}

// PF_KERNEL_AUTO takes this pass where it measured faster than the two-pass
// kernels on MI355X: float32 state with more than 8 flows (per iteration:
// DAGMF 256x512x512 9.63 against 10.86 ms, HMF 128x256x256 0.826 against
// 0.841 ms; the 7-flow Ishikawa chain 0.637 against 0.625 ms).  With 16-bit
// state the two-pass kernels stay ahead (DAGMF bf16 6.59 against 5.62 ms):
// this pass is bound by its instruction latency at one block per compute
// unit, the two-pass kernels by memory bandwidth.
bool flow_label_preferred(int nd, int nl, int nn, bool identity, int storage) {
    return storage == PF_FP32 && nn > 8 && flow_label_supported(nd, nl, nn, identity);
}

// About four blocks per compute unit over the pass, chunks of at least 16
// planes (each chunk recomputes one flow plane below it).
FusedGeom flow_label_geometry(const StepArgs &a) { return tile_geometry(a, GX, GY, 1024); }

hipError_t launch_flow_label(const StepArgs &a, int storage, hipStream_t s) {
    if (!flow_label_supported(3, a.nl, a.nn, false) || a.nz < 1) return hipErrorInvalidValue;
    const FusedGeom g = flow_label_geometry(a);
    if (g.blocks <= 0 || g.blocks > 0x7fffffffL) return hipErrorInvalidValue;
    auto go = [&]<int NL, int NN, typename T>() {
        k_flow_label<NL, NN, T><<<(unsigned)g.blocks, GTHREADS, 0, s>>>(a, g);
        return hipGetLastError();
    };
    auto by = [&]<typename T>() -> hipError_t {
        if (a.nl <= 4 && a.nn <= 8) return go.template operator()<4, 8, T>();
        if (a.nl <= 8 && a.nn <= 8) return go.template operator()<8, 8, T>();
        if (a.nl <= 8 && a.nn <= 12) return go.template operator()<8, 12, T>();
        if (a.nl <= 8 && a.nn <= 16) return go.template operator()<8, 16, T>();
        if (a.nl <= 12 && a.nn <= 16) return go.template operator()<12, 16, T>();
        return go.template operator()<16, 16, T>();
    };
    if (storage == PF_BF16) return by.template operator()<bf16s>();
    if (storage == PF_FP16) return by.template operator()<f16s>();
    return by.template operator()<float>();
}

}  // namespace pf
