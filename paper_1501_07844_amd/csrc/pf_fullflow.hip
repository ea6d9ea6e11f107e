// Full-flow continuous max-flow for the Potts model on gfx950: the method
// the pseudo-flow representation replaces, kept to measure what it saves
// (the paper's Potts primal max-flow and primal-dual models, section
// "Pseudo-Flow Approach to the Potts Model"; its memory claims in the
// abstract and after Algorithm 2).
//
// Every variable of the primal-dual model is explicit: the spatial flows q_L,
// the source flow p_S, the sink flows p_L <= D_L and the labels u_L (the
// multipliers of flow conservation div q_L - p_S + p_L = 0).  One iteration
// maximises the augmented Lagrangian (penalty c) block by block and then
// takes one multiplier step:
//   flow pass:  q_L <- Proj_{|q_L| <= S_L}(q_L + tau grad w_L)
//   rest pass:  p_L = min(D_L, p_S - div q_L + u_L / c)
//               p_S <- (1/n) sum_L (div q_L + p_L - u_L / c) + 1 / (n c)
//               u_L <- u_L - c (div q_L - p_S + p_L)
//               w_L <- div q_L - p_S + p_L - u_L / c
// with w_L the flow step's driver at the start of the next iteration; storing
// it instead of p_L keeps the state at q, u, w and p_S: (nd + 2) n + 1 fields
// per voxel against the pseudo-flow method's (nd + 1) n.  The grid operators
// (forward gradient with a zero last index, divergence as its negative
// adjoint, Euclidean projection) are those of the pseudo-flow kernels.  Both
// passes are elementwise plus nearest-neighbour stencils, in place (each
// writes only fields the other neighbours do not read in that pass), one
// voxel per lane.

#include <hip/hip_runtime.h>
#include <math.h>

#include "pf_device.h"
#include "pf_fullflow.h"
#include "pf_internal.h"

namespace pf {
namespace {

using namespace dev;

// Element L of a [B][F][V] float field at voxel offset uv (uniform base, the
// voxel as a 32-bit offset).
__device__ __forceinline__ const float *fbase(const float *p, int b, int nf, int f, size_t V) {
    return p + ((size_t)b * nf + f) * V;
}
__device__ __forceinline__ float *fbase_w(float *p, int b, int nf, int f, size_t V) {
    return p + ((size_t)b * nf + f) * V;
}

template <int ND, int NLMAX>
__global__ __launch_bounds__(kBlock) void k_ff_init(StepArgs a, FFArgs f) {
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= a.V) return;
    const int b = blockIdx.y;
    const size_t V = (size_t)a.V;
    const unsigned uv = (unsigned)v;
    float m = INFINITY;
#pragma unroll
    for (int L = 0; L < NLMAX; ++L)
        if (L < a.nl) m = fminf(m, ldf(fbase(a.D, b, a.nl, L, V), uv));
    sto(fbase_w(f.pS, b, 1, 0, V), uv, m);
    const float u0 = 1.0f / (float)a.nl;
    // w = div q - p_S + p_L - u / c with q = 0 and p_L = p_S
    const float w0 = ((0.f - m) + m) - u0 * a.inv_c;
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        if (L < a.nl) {
            sto(fbase_w(f.u, b, a.nl, L, V), uv, u0);
            sto(fbase_w(f.w, b, a.nl, L, V), uv, w0);
#pragma unroll
            for (int k = 0; k < ND; ++k) sto(fbase_w(f.q, b, a.nl * ND, L * ND + k, V), uv, 0.f);
        }
    }
}

// Spatial flows: q_L <- Proj(q_L + tau grad w_L), component k 0 on the last
// index of axis k.
template <int ND, int NLMAX>
__global__ __launch_bounds__(kBlock) void k_ff_flow(StepArgs a, FFArgs f) {
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= a.V) return;
    const int b = blockIdx.y;
    const Coord c = coord_of(v, a.nx, a.ny);
    const size_t V = (size_t)a.V;
    const unsigned uv = (unsigned)v;
    const bool h[3] = {c.x < a.nx - 1, c.y < a.ny - 1, ND == 3 && c.z < a.nz - 1};
    const unsigned off[3] = {h[0] ? 1u : 0u, h[1] ? (unsigned)a.nx : 0u,
                             h[2] ? (unsigned)(a.nx * a.ny) : 0u};
    // load phase: unconditional, label index clamped
    float w0[NLMAX], wn[NLMAX][ND], qv[NLMAX][ND], sv[NLMAX];
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        const int Lc = L < a.nl ? L : a.nl - 1;
        const float *wb = fbase(f.w, b, a.nl, Lc, V);
        w0[L] = ldf(wb, uv);
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            wn[L][k] = ldf(wb, uv + off[k]);
            qv[L][k] = ldf(fbase(f.q, b, a.nl * ND, Lc * ND + k, V), uv);
        }
        sv[L] = smooth(a, b, Lc, v);
    }
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        if (L < a.nl) {
            float p[ND];
            float n2 = 0.f;
#pragma unroll
            for (int k = 0; k < ND; ++k) {
                p[k] = h[k] ? fmaf(f.tau, wn[L][k] - w0[L], qv[L][k]) : 0.f;
                n2 = fmaf(p[k], p[k], n2);
            }
            const float S = sv[L];
            if (n2 > S * S) {
                const float sc = S * rsqrtf(n2);
#pragma unroll
                for (int k = 0; k < ND; ++k) p[k] *= sc;
            }
#pragma unroll
            for (int k = 0; k < ND; ++k) sto(fbase_w(f.q, b, a.nl * ND, L * ND + k, V), uv, p[k]);
        }
    }
}

// Sink flows, source flow, labels, and the next flow driver, at one voxel.
template <int ND, int NLMAX>
__global__ __launch_bounds__(kBlock) void k_ff_rest(StepArgs a, FFArgs f) {
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
    float q0[NLMAX][3], qm[NLMAX][3], uu[NLMAX], dd[NLMAX];
    const float ps = ldf(fbase(f.pS, b, 1, 0, V), uv);
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        const int Lc = L < a.nl ? L : a.nl - 1;
        uu[L] = ldf(fbase(f.u, b, a.nl, Lc, V), uv);
        dd[L] = ldf(fbase(a.D, b, a.nl, Lc, V), uv);
        q0[L][2] = qm[L][2] = 0.f;
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            const float *qb = fbase(f.q, b, a.nl * ND, Lc * ND + k, V);
            q0[L][k] = ldf(qb, uv);
            qm[L][k] = ldf(qb, uv - (unsigned)m[k]);
        }
    }
    float dq[NLMAX], pl[NLMAX];
    float acc = 0.f;
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        dq[L] = div_from<ND>(q0[L], qm[L], fwd, bwd);
        pl[L] = fminf(dd[L], (ps - dq[L]) + uu[L] * a.inv_c);
        if (L < a.nl) acc += (dq[L] + pl[L]) - uu[L] * a.inv_c;
    }
    const float inv_n = 1.0f / (float)a.nl;
    const float ps1 = fmaf(acc, inv_n, inv_n * a.inv_c);
    sto(fbase_w(f.pS, b, 1, 0, V), uv, ps1);
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        if (L < a.nl) {
            const float r = (dq[L] - ps1) + pl[L];
            const float u1 = fmaf(-f.c, r, uu[L]);
            sto(fbase_w(f.u, b, a.nl, L, V), uv, u1);
            sto(fbase_w(f.w, b, a.nl, L, V), uv, r - u1 * a.inv_c);
        }
    }
}

// u clipped at 0 and renormalised over the labels (uniform where all clip).
template <int NLMAX>
__device__ __forceinline__ void feasible(const float (&u)[NLMAX], int n, double (&t)[NLMAX]) {
    double s = 0.0;
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        t[L] = L < n ? fmax((double)u[L], 0.0) : 0.0;
        s += t[L];
    }
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) t[L] = s > 0.0 ? t[L] / s : (L < n ? 1.0 / n : 0.0);
}

// float64 energy of the feasible labels, pseudo-flow dual of q, max
// |sum u - 1|, max |q| - S; one partial per block, a fixed-order tree.
template <int ND, int NLMAX>
__global__ __launch_bounds__(kBlock) void k_ff_energy(StepArgs a, FFArgs f, double *partials) {
    __shared__ double red[4][kBlock];
    const size_t V = (size_t)a.V;
    const size_t total = V * (size_t)a.B;
    double e_sum = 0.0, p_sum = 0.0, mx_s = 0.0, mx_q = -INFINITY;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (size_t)gridDim.x * kBlock) {
        const int b = (int)(i / V);
        const int v = (int)(i - (size_t)b * V);
        const unsigned uv = (unsigned)v;
        const Coord c = coord_of(v, a.nx, a.ny);
        int m[3];
        bool bwd[3];
        backward_offsets(c, a, m, bwd);
        const bool h[3] = {c.x < a.nx - 1, c.y < a.ny - 1, ND == 3 && c.z < a.nz - 1};
        const unsigned off[3] = {h[0] ? 1u : 0u, h[1] ? (unsigned)a.nx : 0u,
                                 h[2] ? (unsigned)(a.nx * a.ny) : 0u};
        float u0[NLMAX], un[ND][NLMAX], dl[NLMAX], q0[NLMAX][3], qm[NLMAX][3], sv[NLMAX];
#pragma unroll
        for (int L = 0; L < NLMAX; ++L) {
            const int Lc = L < a.nl ? L : a.nl - 1;
            const float *ub = fbase(f.u, b, a.nl, Lc, V);
            u0[L] = ldf(ub, uv);
#pragma unroll
            for (int k = 0; k < ND; ++k) un[k][L] = ldf(ub, uv + off[k]);
            dl[L] = ldf(fbase(a.D, b, a.nl, Lc, V), uv);
            q0[L][2] = qm[L][2] = 0.f;
#pragma unroll
            for (int k = 0; k < ND; ++k) {
                const float *qb = fbase(f.q, b, a.nl * ND, Lc * ND + k, V);
                q0[L][k] = ldf(qb, uv);
                qm[L][k] = ldf(qb, uv - (unsigned)m[k]);
            }
            sv[L] = smooth(a, b, Lc, v);
        }
        double t0[NLMAX], tn[ND][NLMAX];
        feasible<NLMAX>(u0, a.nl, t0);
#pragma unroll
        for (int k = 0; k < ND; ++k) feasible<NLMAX>(un[k], a.nl, tn[k]);
        double e = 0.0, pm = INFINITY, su = 0.0;
#pragma unroll
        for (int L = 0; L < NLMAX; ++L) {
            if (L < a.nl) {
                const double S = (double)sv[L];
                double g2 = 0.0, qn2 = 0.0, dv = 0.0;
#pragma unroll
                for (int k = 0; k < ND; ++k) {
                    const double g = h[k] ? tn[k][L] - t0[L] : 0.0;
                    g2 += g * g;
                    qn2 += (double)q0[L][k] * (double)q0[L][k];
                    dv += h[k] ? (double)q0[L][k] : 0.0;
                    dv -= bwd[k] ? (double)qm[L][k] : 0.0;
                }
                e += (double)dl[L] * t0[L] + S * sqrt(g2);
                pm = fmin(pm, (double)dl[L] + dv);
                mx_q = fmax(mx_q, sqrt(qn2) - S);
                su += (double)u0[L];
            }
        }
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

// Fixed-order reduction of the block partials (sums of slots 0 and 1, maxima
// of slots 2 and 3).
__global__ __launch_bounds__(kBlock) void k_ff_reduce(const double *partials, int n,
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
    if (threadIdx.x == 0)
        for (int j = 0; j < 4; ++j) results[j] = red[j][0];
}

// u (the multipliers as they are), the argmax labels (ties: lowest) and q.
template <int ND, int NLMAX>
__global__ __launch_bounds__(kBlock) void k_ff_export(StepArgs a, FFArgs f, float *u,
                                                      int32_t *labels, float *q) {
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= a.V) return;
    const int b = blockIdx.y;
    const size_t V = (size_t)a.V;
    const unsigned uv = (unsigned)v;
    float best = -INFINITY;
    int arg = 0;
    for (int L = 0; L < a.nl; ++L) {
        const float x = ldf(fbase(f.u, b, a.nl, L, V), uv);
        if (u) sto(fbase_w(u, b, a.nl, L, V), uv, x);
        if (x > best) {
            best = x;
            arg = L;
        }
        if (q) {
            for (int k = 0; k < ND; ++k)
                sto(fbase_w(q, b, a.nl * ND, L * ND + k, V), uv,
                    ldf(fbase(f.q, b, a.nl * ND, L * ND + k, V), uv));
        }
    }
    if (labels) labels[(size_t)b * V + v] = arg;
}

// ----------------------------------------------------------- dispatch ----

template <typename F>
hipError_t ff_dispatch(int nd, int n, F &&fn) {
    auto by = [&]<int ND>() -> hipError_t {
        if (n <= 4) return fn.template operator()<ND, 4>();
        if (n <= 8) return fn.template operator()<ND, 8>();
        return fn.template operator()<ND, 16>();
    };
    return nd == 2 ? by.template operator()<2>() : by.template operator()<3>();
}

dim3 ff_grid(const StepArgs &a) {
    return dim3((unsigned)((a.V + kBlock - 1) / kBlock), (unsigned)a.B, 1);
}

}  // namespace

bool ff_supported(int nd, int n) { return (nd == 2 || nd == 3) && n >= 1 && n <= 16; }

static size_t ff_align(size_t x) { return (x + 255) & ~size_t(255); }

FFLayout ff_layout(const pf_grid &g, int n) {
    FFLayout L{};
    const size_t V = (size_t)g.nx * g.ny * g.nz, B = (size_t)g.batch;
    size_t off = 0;
    L.results = off;
    off += 256;
    L.partials = off;
    off = ff_align(off + (size_t)kPartials * 4 * sizeof(double));
    L.consts = off;
    off = ff_align(off + sizeof(ConstBlock));
    L.q = off;
    off = ff_align(off + B * n * g.ndim * V * 4);
    L.u = off;
    off = ff_align(off + B * n * V * 4);
    L.w = off;
    off = ff_align(off + B * n * V * 4);
    L.pS = off;
    off = ff_align(off + B * V * 4);
    L.total = off;
    return L;
}

hipError_t launch_ff_init(const StepArgs &a, const FFArgs &f, int nd, hipStream_t s) {
    return ff_dispatch(nd, a.nl, [&]<int ND, int NL>() {
        k_ff_init<ND, NL><<<ff_grid(a), kBlock, 0, s>>>(a, f);
        return hipGetLastError();
    });
}

hipError_t launch_ff_iteration(const StepArgs &a, const FFArgs &f, int nd, hipStream_t s) {
    return ff_dispatch(nd, a.nl, [&]<int ND, int NL>() {
        k_ff_flow<ND, NL><<<ff_grid(a), kBlock, 0, s>>>(a, f);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        k_ff_rest<ND, NL><<<ff_grid(a), kBlock, 0, s>>>(a, f);
        return hipGetLastError();
    });
}

hipError_t launch_ff_energy(const StepArgs &a, const FFArgs &f, int nd, double *partials,
                            double *results, hipStream_t s) {
    hipError_t e = ff_dispatch(nd, a.nl, [&]<int ND, int NL>() {
        k_ff_energy<ND, NL><<<kPartials, kBlock, 0, s>>>(a, f, partials);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    k_ff_reduce<<<1, kBlock, 0, s>>>(partials, kPartials, results);
    return hipGetLastError();
}

hipError_t launch_ff_export(const StepArgs &a, const FFArgs &f, int nd, float *u, int32_t *labels,
                            float *q, hipStream_t s) {
    return ff_dispatch(nd, a.nl, [&]<int ND, int NL>() {
        k_ff_export<ND, NL><<<ff_grid(a), kBlock, 0, s>>>(a, f, u, labels, q);
        return hipGetLastError();
    });
}

}  // namespace pf
