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
// KA reads lbar at x and x + e_k, KB reads pbar at x and x - e_k, so each is
// its own launch; both update their buffers in place (a thread writes only
// its own voxel).

#include <hip/hip_runtime.h>
#include <math.h>

#include "pf_device.h"
#include "pf_internal.h"

namespace pf {
namespace {

using namespace dev;

template <int ND, int NLMAX, int NNMAX, bool IDENT>
__global__ __launch_bounds__(kBlock) void k_adj_flow(StepArgs a, AdjArgs g) {
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= a.V) return;
    const int b = blockIdx.y;
    const Coord c = coord_of(v, a.nx, a.ny);
    const size_t V = (size_t)a.V;
    const unsigned uv = (unsigned)v;
    const bool h[3] = {c.x < a.nx - 1, c.y < a.ny - 1, ND == 3 && c.z < a.nz - 1};
    const int off[3] = {h[0] ? 1 : 0, h[1] ? a.nx : 0, h[2] ? a.nx * a.ny : 0};

    // loads: new labels (x and forward neighbours), lbar (same), old flows,
    // pbar of the later step, capacities
    float e0[NLMAX], en[NLMAX][ND], l0[NLMAX], lnb[NLMAX][ND];
    float qv[NNMAX][ND], pb[NNMAX][ND], sv[NNMAX];
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        const int Lc = L < a.nl ? L : a.nl - 1;
        const float *el = field<float>(g.ell_next, b, a.nl, Lc, V);
        const float *lb = field<float>(g.lbar, b, a.nl, Lc, V);
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
            pb[A][k] = ldf(field<float>(g.pbar, b, a.nn * ND, Ac * ND + k, V), uv);
        }
        sv[A] = smooth(a, b, Ac, v);
    }
    // forward quantities: grad u', grad U, p
    float gu[NLMAX][ND], gl[NLMAX][ND];
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        const float u0 = __expf(e0[L]);
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            gu[L][k] = h[k] ? __expf(en[L][k]) - u0 : 0.f;
            gl[L][k] = h[k] ? lnb[L][k] - l0[L] : 0.f;      // grad of lbar
        }
    }
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) {
        if (A < a.nn) {
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
            float out[ND], sbar = 0.f;
            if (n2 > S * S) {
                const float rn = rsqrtf(n2);
                const float sc = S * rn;
                const float proj = dot / n2;
#pragma unroll
                for (int k = 0; k < ND; ++k) out[k] = sc * (qb[k] - proj * p[k]);
                sbar = dot * rn;
            } else {
#pragma unroll
                for (int k = 0; k < ND; ++k) out[k] = qb[k];
            }
#pragma unroll
            for (int k = 0; k < ND; ++k) {
                float *po = field_w<float>(g.pbar, b, a.nn * ND, A * ND + k, V);
                *reinterpret_cast<float *>(reinterpret_cast<char *>(po) + uv * 4u) =
                    h[k] ? out[k] : 0.f;
            }
            float *sb = field_w<float>(g.sbar, b, a.nn, A, V);
            float *sp = reinterpret_cast<float *>(reinterpret_cast<char *>(sb) + uv * 4u);
            *sp += sbar;
        }
    }
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

    float e[NLMAX], lb[NLMAX], p0[NNMAX][3], pm[NNMAX][3];
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        const int Lc = L < a.nl ? L : a.nl - 1;
        e[L] = ldf(field<float>(g.ell_next, b, a.nl, Lc, V), uv);
        lb[L] = ldf(field<float>(g.lbar, b, a.nl, Lc, V), uv);
    }
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) {
        const int Ac = A < a.nn ? A : a.nn - 1;
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            const float *pk = field<float>(g.pbar, b, a.nn * ND, Ac * ND + k, V);
            p0[A][k] = ldf(pk, uv);
            pm[A][k] = ldf(pk, uv - (unsigned)m[k]);
        }
    }
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
    float gt[NLMAX], sg = 0.f;
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        const float u = __expf(e[L]);
        gt[L] = L < a.nl ? fmaf(ub[L], u, lb[L]) : 0.f;
        sg += gt[L];
    }
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        if (L < a.nl) {
            const float tb = gt[L] - __expf(e[L]) * sg;
            float *lo = field_w<float>(g.lbar, b, a.nl, L, V);
            *reinterpret_cast<float *>(reinterpret_cast<char *>(lo) + uv * 4u) = tb;
            float *dd = field_w<float>(g.dbar, b, a.nl, L, V);
            float *dp = reinterpret_cast<float *>(reinterpret_cast<char *>(dd) + uv * 4u);
            *dp -= tb * a.inv_c;
        }
    }
}

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

// dS for a shared field: sum over nodes at every voxel.
__global__ __launch_bounds__(kBlock) void k_sum_over_nodes(const float *sbar, int nn, size_t V,
                                                           float *out) {
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if ((size_t)v >= V) return;
    const int b = blockIdx.y;
    float s = 0.f;
    for (int A = 0; A < nn; ++A) s += sbar[((size_t)b * nn + A) * V + v];
    out[(size_t)b * V + v] = s;
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

}  // namespace

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

hipError_t launch_reduce_sbar(const float *sbar, int B, int nn, size_t V, int s_mode, float *out,
                              hipStream_t s) {
    if (s_mode == PF_S_NODE_SCALAR) {
        k_sum_nodes<<<nn, kBlock, 0, s>>>(sbar, B, nn, V, out);
    } else if (s_mode == PF_S_SHARED_FIELD) {
        k_sum_over_nodes<<<dim3((unsigned)((V + kBlock - 1) / kBlock), (unsigned)B), kBlock, 0, s>>>(
            sbar, nn, V, out);
    } else {
        return launch_copy_f(sbar, out, (size_t)B * nn * V, s);
    }
    return hipGetLastError();
}

}  // namespace pf
