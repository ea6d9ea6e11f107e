// Device helpers shared by the iteration kernels (pf_kernels.hip and
// pf_fused.hip), so that the two-pass and the fused single-pass kernels
// evaluate the same float32 expressions in the same order.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "pf_internal.h"

namespace pf {
namespace dev {

// ------------------------------------------------------------ storage ----

struct bf16s {
    uint16_t b;
};
using f16s = _Float16;

__device__ __forceinline__ float ld(const float *p, size_t i) { return p[i]; }
__device__ __forceinline__ float ld(const bf16s *p, size_t i) {
    return __uint_as_float(uint32_t(p[i].b) << 16);
}
__device__ __forceinline__ float ld(const f16s *p, size_t i) { return (float)p[i]; }

// float -> bf16 bits, round to nearest even (gfx950 converts in hardware:
// v_cvt_pk_bf16_f32, two values per instruction)
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_bits(float v) {
    const __bf16 h = (__bf16)v;
    uint16_t r;
    __builtin_memcpy(&r, &h, 2);
    return r;
}
__device__ __forceinline__ uint32_t f16_bits(float v) {
    const f16s h = (f16s)v;
    uint16_t r;
    __builtin_memcpy(&r, &h, 2);
    return r;
}

__device__ __forceinline__ void st(float *p, size_t i, float v) { p[i] = v; }
__device__ __forceinline__ void st(bf16s *p, size_t i, float v) { p[i].b = uint16_t(bf16_bits(v)); }
__device__ __forceinline__ void st(f16s *p, size_t i, float v) { p[i] = (f16s)v; }

// Per-solve constants (node capacities, path weights) live in the workspace
// and are read through the constant address space: uniform across the
// wavefront and never written by the iteration kernels, so they become
// scalar loads.
using cfloat = const __attribute__((address_space(4))) float;
__device__ __forceinline__ float cld(const float *p, int i) {
    return ((cfloat *)p)[i];
}
__device__ __forceinline__ float wgt(const StepArgs &a, int A, int L) {
    return cld(a.W, A * PF_MAX_LEAVES + L);
}

// ------------------------------------------------------------ helpers ----

// Start of field f of problem b in a [B][F][V] array: uniform across the
// block, so that loads become "uniform base + 32-bit lane offset" (the
// global saddr form, one offset VGPR shared by every field of a voxel).
// N32 forms the field index b*F + f in 32 bits (B*F is far below 2^31) and
// widens it once for the product with V; the result is the same, the scalar
// code differs (N32 measured faster in the two-iteration kernel and slower in
// the one-iteration one, so each kernel picks its form).
template <typename T, bool N32 = false>
__device__ __forceinline__ const T *field(const void *base, int b, int nf, int f, size_t V) {
    if constexpr (N32) return static_cast<const T *>(base) + (size_t)(uint32_t)(b * nf + f) * V;
    return static_cast<const T *>(base) + ((size_t)b * nf + f) * V;
}
template <typename T, bool N32 = false>
__device__ __forceinline__ T *field_w(void *base, int b, int nf, int f, size_t V) {
    if constexpr (N32) return static_cast<T *>(base) + (size_t)(uint32_t)(b * nf + f) * V;
    return static_cast<T *>(base) + ((size_t)b * nf + f) * V;
}

// Load / store at a 32-bit byte offset from a uniform base.  Voxels per
// problem are capped at 2^30 by the host checks, so offsets of 4-byte
// fields fit in 32 bits; the explicit 32-bit offset lets the compiler use
// one shared offset VGPR with the base in SGPRs.
template <typename T>
__device__ __forceinline__ float ldo(const T *base, unsigned idx) {
    return ld(reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                          (unsigned)(idx * (unsigned)sizeof(T))), 0);
}
template <typename T>
__device__ __forceinline__ void sto(T *base, unsigned idx, float v) {
    st(reinterpret_cast<T *>(reinterpret_cast<char *>(base) + (unsigned)(idx * (unsigned)sizeof(T))),
       0, v);
}
__device__ __forceinline__ float ldf(const float *base, unsigned idx) {
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + idx * 4u);
}

// ------------------------------------------------------ state layout ----
// fp32 state: one float per field and voxel, ell [B][nl][V], q [B][nn][nd][V].
// 16-bit state: fields packed in pairs into 32-bit words, so that every state
// load and store is an aligned dword: ell [B][ceil(nl/2)][V] words holding
// labels (2P, 2P+1), q [B][ceil(nn/2)][nd][V] words holding component k of
// flows (2P, 2P+1).  The neighbour of a voxel in any axis is the same word at
// another voxel.  The spare half of an odd count is written as 0 by every
// store (the initialisation writes ell0 there).
template <typename T>
inline constexpr bool kPacked = sizeof(T) == 2;

__device__ __forceinline__ float half_of(uint32_t w, int h, const bf16s *) {
    return __uint_as_float(h ? (w & 0xffff0000u) : (w << 16));
}
__device__ __forceinline__ float half_of(uint32_t w, int h, const f16s *) {
    const uint16_t r = uint16_t(h ? (w >> 16) : (w & 0xffffu));
    f16s x;
    __builtin_memcpy(&x, &r, 2);
    return (float)x;
}
__device__ __forceinline__ uint32_t pack2(float lo, float hi, const bf16s *) {
    const f32x2_t v = {lo, hi};
    const bf16x2_t h = __builtin_convertvector(v, bf16x2_t);
    uint32_t w;
    __builtin_memcpy(&w, &h, 4);
    return w;
}
__device__ __forceinline__ uint32_t pack2(float lo, float hi, const f16s *) {
    return f16_bits(lo) | (f16_bits(hi) << 16);
}

// Label L of problem b at voxel index uv.  L past the last label reads a
// valid field (clamped; the caller masks it), and the clamp is taken on the
// word index for packed state, so that L = 2P and 2P + 1 load the same word
// and the compiler merges the two loads.
template <typename T, bool N32 = false>
__device__ __forceinline__ float ld_ell(const void *base, int b, int nl, int L, size_t V, unsigned uv) {
    if constexpr (kPacked<T>) {
        const int np = (nl + 1) / 2, P = L >> 1;
        const uint32_t *p = field<uint32_t, N32>(base, b, np, P < np ? P : np - 1, V);
        const uint32_t w = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(p) + uv * 4u);
        return half_of(w, L & 1, static_cast<const T *>(nullptr));
    } else {
        return ldf(field<float, N32>(base, b, nl, L < nl ? L : nl - 1, V), uv);
    }
}

// Component k of flow A of problem b at voxel index uv (A clamped as L above).
template <typename T, int ND, bool N32 = false>
__device__ __forceinline__ float ld_q(const void *base, int b, int nn, int A, int k, size_t V,
                                      unsigned uv) {
    if constexpr (kPacked<T>) {
        const int np = (nn + 1) / 2, P = A >> 1;
        const uint32_t *p = field<uint32_t, N32>(base, b, np * ND, (P < np ? P : np - 1) * ND + k, V);
        const uint32_t w = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(p) + uv * 4u);
        return half_of(w, A & 1, static_cast<const T *>(nullptr));
    } else {
        return ldf(field<float, N32>(base, b, nn * ND, (A < nn ? A : nn - 1) * ND + k, V), uv);
    }
}

// Labels L and L + 1 (L even) at voxel uv; nothing past nl is stored (a
// packed word's spare half gets 0).
template <typename T, bool N32 = false>
__device__ __forceinline__ void st_ell2(void *base, int b, int nl, int L, size_t V, unsigned uv,
                                        float lo, float hi) {
    if constexpr (kPacked<T>) {
        if (L < nl) {
            uint32_t *p = field_w<uint32_t, N32>(base, b, (nl + 1) / 2, L >> 1, V);
            *reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(p) + uv * 4u) =
                pack2(lo, L + 1 < nl ? hi : 0.f, static_cast<const T *>(nullptr));
        }
    } else {
        if (L < nl) sto(field_w<float, N32>(base, b, nl, L, V), uv, lo);
        if (L + 1 < nl) sto(field_w<float, N32>(base, b, nl, L + 1, V), uv, hi);
    }
}

// Component k of flows A and A + 1 (A even) at voxel uv.
template <typename T, int ND, bool N32 = false>
__device__ __forceinline__ void st_q2(void *base, int b, int nn, int A, int k, size_t V,
                                      unsigned uv, float lo, float hi) {
    if constexpr (kPacked<T>) {
        if (A < nn) {
            uint32_t *p = field_w<uint32_t, N32>(base, b, (nn + 1) / 2 * ND, (A >> 1) * ND + k, V);
            *reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(p) + uv * 4u) =
                pack2(lo, A + 1 < nn ? hi : 0.f, static_cast<const T *>(nullptr));
        }
    } else {
        if (A < nn) sto(field_w<float, N32>(base, b, nn * ND, A * ND + k, V), uv, lo);
        if (A + 1 < nn) sto(field_w<float, N32>(base, b, nn * ND, (A + 1) * ND + k, V), uv, hi);
    }
}

struct Coord {
    int x, y, z;
};

__device__ __forceinline__ Coord coord_of(int v, int nx, int ny) {
    Coord c;
    c.x = v % nx;
    const int r = v / nx;
    c.y = r % ny;
    c.z = r / ny;
    return c;
}

// S_A at voxel v of problem b, one strided load for every s_mode.  (A
// three-way branch on s_mode here was miscompiled by hipcc 7.2 in the fully
// unrolled weighted fp64 reduction: on the per-node-field path the node index
// feeding the following flow address was read from a register that path never
// wrote.  The branch-free form leaves no such path.)
__device__ __forceinline__ float smooth(const StepArgs &a, int b, int A, int v) {
    const float *base = a.Sp + ((int64_t)b * a.s_sb + (int64_t)A * a.s_sa);
    return ldf(base, (unsigned)v * (unsigned)a.s_sv);
}

// div q_A from the flow components at x (q0) and at x - e_k (qm):
// sum_k q_k(x)[x_k < N_k - 1] - q_k(x - e_k)[x_k > 0].  Selects, no branches.
template <int ND>
__device__ __forceinline__ float div_from(const float (&q0)[3], const float (&qm)[3],
                                          const bool (&fwd)[3], const bool (&bwd)[3]) {
    float dv = 0.f;
#pragma unroll
    for (int k = 0; k < ND; ++k) {
        dv += fwd[k] ? q0[k] : 0.f;
        dv -= bwd[k] ? qm[k] : 0.f;
    }
    return dv;
}

// Offsets of the backward neighbours, 0 on the first index of an axis so
// that the (unconditional) load stays inside the volume.
__device__ __forceinline__ void backward_offsets(const Coord &c, const StepArgs &a, int (&m)[3],
                                                 bool (&bwd)[3]) {
    bwd[0] = c.x > 0;
    bwd[1] = c.y > 0;
    bwd[2] = c.z > 0;
    m[0] = bwd[0] ? 1 : 0;
    m[1] = bwd[1] ? a.nx : 0;
    m[2] = bwd[2] ? a.nx * a.ny : 0;
}

// Value after a round trip through the storage type (what a later load of a
// stored value returns).
__device__ __forceinline__ float roundtrip(float v, const float *) { return v; }
__device__ __forceinline__ float roundtrip(float v, const bf16s *) {
    bf16s t;
    st(&t, 0, v);
    return ld(&t, 0);
}
__device__ __forceinline__ float roundtrip(float v, const f16s *) { return (float)(f16s)v; }

// Projected gradient step of one flow at one voxel:
// p = q - c tau G (component k forced to 0 where x_k is the last index),
// then p * min(1, S / |p|).
template <int ND>
__device__ __forceinline__ void flow_project(const StepArgs &a, const float (&q)[ND],
                                             const float (&G)[3], const bool (&h)[3], float S,
                                             float (&p)[ND]) {
#pragma unroll
    for (int k = 0; k < ND; ++k) p[k] = h[k] ? fmaf(-a.ctau, G[k], q[k]) : 0.f;
    float n2 = 0.f;
#pragma unroll
    for (int k = 0; k < ND; ++k) n2 = fmaf(p[k], p[k], n2);
    if (n2 > S * S) {
        const float sc = S * rsqrtf(n2);
#pragma unroll
        for (int k = 0; k < ND; ++k) p[k] *= sc;
    }
}

// Top-down flow excess in path-weight form: d_L += W[A][L] * div q_A
// (identity for Potts).  W is zero for nodes and leaves outside the graph,
// so no guards are needed.
template <int NLMAX, bool IDENT>
__device__ __forceinline__ void add_excess(const StepArgs &a, float (&d)[NLMAX], int A, float dv) {
    if constexpr (IDENT) {
        d[A] += dv;
    } else {
#pragma unroll
        for (int L = 0; L < NLMAX; ++L) d[L] = fmaf(wgt(a, A, L), dv, d[L]);
    }
}

// grad U_A = sum_L W[A][L] grad u_L (identity for Potts).
template <int ND, int NLMAX, bool IDENT>
__device__ __forceinline__ void grad_U(const StepArgs &a, int A, const float (&gu)[NLMAX][ND],
                                       float (&G)[3]) {
    G[0] = G[1] = G[2] = 0.f;
    if constexpr (IDENT) {
#pragma unroll
        for (int k = 0; k < ND; ++k) G[k] = gu[A][k];
    } else {
#pragma unroll
        for (int L = 0; L < NLMAX; ++L) {
            const float w = wgt(a, A, L);
#pragma unroll
            for (int k = 0; k < ND; ++k) G[k] = fmaf(w, gu[L][k], G[k]);
        }
    }
}

// Entropic proximal (Bregman) label step in the log domain:
// ell_L <- (t_L - m) - ln sum_L' exp(t_L' - m),  t_L = ell_L - d_L / c,  m = max t.
// Slots L >= nl hold copies of a valid label and are masked to -inf.
template <int NLMAX>
__device__ __forceinline__ void entropic_step(const StepArgs &a, const float (&d)[NLMAX],
                                              float (&ell)[NLMAX]) {
    float m = -INFINITY;
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        ell[L] = L < a.nl ? fmaf(-d[L], a.inv_c, ell[L]) : -INFINITY;
        m = fmaxf(m, ell[L]);
    }
    float s = 0.f;
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) s += __expf(ell[L] - m);
    const float ls = __logf(s);
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) ell[L] = (ell[L] - m) - ls;
}

}  // namespace dev
}  // namespace pf
