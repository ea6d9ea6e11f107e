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
constexpr int GY = 8;                      // owned tile rows (4: 1.17-1.32x slower)
constexpr int GTHREADS = GX * (GY + 2);    // owned rows, the halo row, the halo column

// Flow slots of a build: NI dense slots (slot s is node s, its path-weight
// row W[s][*] read from the constants), then, when TAIL, NLMAX identity slots:
// slot NI + L is node ni + L with ni = nn - nl, the end-label L itself, whose
// row is the unit vector of L.  The host takes TAIL only for graphs whose
// last nl nodes are the end-labels in order (every internal node numbered
// before every leaf), and with 16-bit state only for an even ni (a packed
// pair of flows never straddles the two kinds).  An identity slot's grad U is
// grad u_L and its excess goes to d_L alone: the values the dense products
// give (every other term is an exact zero), without the products.  EXACT
// builds serve graphs that fill every slot (nl = NLMAX, and nn - nl = NI with
// TAIL or nn = NI without): slot s is node s and every slot is valid, known
// at compile time; then a slot pair is a node pair whatever the parity of
// NI, and an odd slot count gets one padding slot (NP), invalid.
template <int NLMAX, int NI, bool TAIL, bool EXACT>
struct Slots {
    static constexpr int N = TAIL ? NI + NLMAX : NI;
    static constexpr int NP = (N + 1) / 2 * 2;
    static __device__ __forceinline__ bool tail(int s) { return TAIL && s >= NI; }
    static __device__ __forceinline__ int node(const StepArgs &a, int s) {
        if constexpr (EXACT) return s;
        return tail(s) ? (a.nn - a.nl) + (s - NI) : s;
    }
    static __device__ __forceinline__ bool valid(const StepArgs &a, int s) {
        if constexpr (EXACT) return s < N;
        return tail(s) ? s - NI < a.nl : s < (TAIL ? a.nn - a.nl : a.nn);
    }
};

// Start of field f (counted over problems and fields) of a [B][F][V] array
// of 4-byte words, formed where it is used from the array's start and a
// field size made opaque by an empty asm statement: otherwise the compiler
// keeps the start of every field the pass touches live across the plane loop
// (about 70 with 16 flows, more than a wavefront's scalar registers) and
// reloads the spilled ones from lanes of a vector register at every use.
__device__ __forceinline__ size_t opaque_size(size_t v) {
    __asm__ volatile("" : "+s"(v));
    return v;
}
template <typename W>
__device__ __forceinline__ const W *fld(const void *base, int f, size_t V) {
    return static_cast<const W *>(base) + (size_t)(unsigned)f * opaque_size(V);
}
template <typename W>
__device__ __forceinline__ W *fld_w(void *base, int f, size_t V) {
    return static_cast<W *>(base) + (size_t)(unsigned)f * opaque_size(V);
}

// Component k of flow A at voxel uv (ld_q with the start formed by fld; A
// clamped into the graph the same way); with 16-bit state the packed word of
// the node pair (A, A + 1), A even, whose halves the caller unpacks (a slot's
// node has the slot's parity: every build's dense count and, with 16-bit
// state, the internal node count are even; a pair past the graph reads some
// valid word, its values unused).  Then the stores of st_q2 / st_ell2.
template <bool EXACT>
__device__ __forceinline__ uint32_t fl_ld_q_word(const StepArgs &a, int b, int A, int k, size_t V,
                                                 unsigned uv) {
    const int np = (a.nn + 1) / 2, P = A >> 1;
    const uint32_t *p = fld<uint32_t>(a.q_in, (b * np + (EXACT || P < np ? P : np - 1)) * 3 + k, V);
    return *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(p) + uv * 4u);
}
__device__ __forceinline__ float fl_ld_q(const StepArgs &a, int b, int A, int k, size_t V, unsigned uv) {
    return ldf(fld<float>(a.q_in, (b * a.nn + (A < a.nn ? A : a.nn - 1)) * 3 + k, V), uv);
}
// (EXACT: A + 1 < nn and L + 1 < nl hold, every build's counts being even)
template <typename T, bool EXACT>
__device__ __forceinline__ void fl_st_q2(const StepArgs &a, int b, int A, int k, size_t V, unsigned uv,
                                         float lo, float hi) {
    if constexpr (kPacked<T>) {
        if (EXACT || A < a.nn) {
            uint32_t *p = fld_w<uint32_t>(a.q_out, (b * ((a.nn + 1) / 2) + (A >> 1)) * 3 + k, V);
            *reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(p) + uv * 4u) =
                pack2(lo, EXACT || A + 1 < a.nn ? hi : 0.f, static_cast<const T *>(nullptr));
        }
    } else {
        if (EXACT || A < a.nn) sto(fld_w<float>(a.q_out, (b * a.nn + A) * 3 + k, V), uv, lo);
        if (EXACT || A + 1 < a.nn) sto(fld_w<float>(a.q_out, (b * a.nn + A + 1) * 3 + k, V), uv, hi);
    }
}
template <typename T, bool EXACT>
__device__ __forceinline__ void fl_st_ell2(const StepArgs &a, int b, int L, size_t V, unsigned uv,
                                           float lo, float hi) {
    if constexpr (kPacked<T>) {
        if (EXACT || L < a.nl) {
            uint32_t *p = fld_w<uint32_t>(a.ell_out, b * ((a.nl + 1) / 2) + (L >> 1), V);
            *reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(p) + uv * 4u) =
                pack2(lo, EXACT || L + 1 < a.nl ? hi : 0.f, static_cast<const T *>(nullptr));
        }
    } else {
        if (EXACT || L < a.nl) sto(fld_w<float>(a.ell_out, b * a.nl + L, V), uv, lo);
        if (EXACT || L + 1 < a.nl) sto(fld_w<float>(a.ell_out, b * a.nl + L + 1, V), uv, hi);
    }
}

// entropic_step (the same expressions in the same order) with the label
// count known at compile time in EXACT builds.
template <int NLMAX, bool EXACT>
__device__ __forceinline__ void fl_entropic_step(const StepArgs &a, const float (&d)[NLMAX],
                                                 float (&ell)[NLMAX]) {
    float m = -INFINITY;
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        ell[L] = EXACT || L < a.nl ? fmaf(-d[L], a.inv_c, ell[L]) : -INFINITY;
        m = fmaxf(m, ell[L]);
    }
    float sum = 0.f;
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) sum += __expf(ell[L] - m);
    const float ls = __logf(sum);
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) ell[L] = (ell[L] - m) - ls;
}

// Flow step of iteration k at voxel (x, y, z): the labels of iteration k at
// the voxel (returned in e0, as stored) and at x + e_k, the old flows at the
// voxel and the capacities; returns the new flows of every slot after a
// round trip through the storage type (what a later load returns; 0 in a
// slot past the graph) and stores them when `store`.
// The Ishikawa chain's path weights are fixed (Algorithm 3): flow j drives
// every label after it, W[j][L] = 1 for L > j and 0 otherwise.  Builds for
// the chain (CH) take them at compile time: grad U_j is the sum of the label
// gradients above j and a flow's divergence adds to the excess of every
// label above it.  These are grad_U's and add_excess's sums with the zero
// terms left out, in the same order, so they give the same values (a term
// fma(0, x, s) leaves a finite sum s unchanged up to the sign of a zero).
// The gradients of padding labels (L >= nl) must be zero.
template <int NLMAX>
__device__ __forceinline__ void grad_U_chain(int A, const float (&gu)[NLMAX][3], float (&G)[3]) {
    G[0] = G[1] = G[2] = 0.f;
#pragma unroll
    for (int L = 0; L < NLMAX; ++L)
        if (L > A)
#pragma unroll
            for (int k = 0; k < 3; ++k) G[k] = fmaf(1.f, gu[L][k], G[k]);
}

template <int NLMAX>
__device__ __forceinline__ void add_excess_chain(float (&d)[NLMAX], int A, float dv) {
#pragma unroll
    for (int L = 0; L < NLMAX; ++L)
        if (L > A) d[L] = fmaf(1.f, dv, d[L]);
}

template <int NLMAX, int NI, bool TAIL, bool EXACT, typename T, bool CH = false>
__device__ __forceinline__ void flow_point(const StepArgs &a, int b, int x, int y, int z, bool store,
                                           float (&e0)[NLMAX],
                                           float (&pr)[Slots<NLMAX, NI, TAIL, EXACT>::NP][3]) {
    using SL = Slots<NLMAX, NI, TAIL, EXACT>;
    constexpr int NS = SL::NP;
    const size_t V = (size_t)a.V;
    const unsigned uv = (unsigned)((z * a.ny + y) * a.nx + x);
    const bool h[3] = {x < a.nx - 1, y < a.ny - 1, z < a.nz - 1};
    const unsigned off[3] = {h[0] ? 1u : 0u, h[1] ? (unsigned)a.nx : 0u,
                             h[2] ? (unsigned)(a.nx * a.ny) : 0u};
    float en[NLMAX][3], qv[NS][3], sv[NS];
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        e0[L] = ld_ell<T>(a.ell_in, b, a.nl, L, V, uv);
#pragma unroll
        for (int k = 0; k < 3; ++k) en[L][k] = ld_ell<T>(a.ell_in, b, a.nl, L, V, uv + off[k]);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int A = SL::valid(a, s) ? SL::node(a, s) : a.nn - 1;
        if constexpr (kPacked<T>) {
            if (s % 2 == 0) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const uint32_t w = fl_ld_q_word<EXACT>(a, b, SL::node(a, s), k, V, uv);
                    qv[s][k] = half_of(w, 0, static_cast<const T *>(nullptr));
                    qv[s + 1][k] = half_of(w, 1, static_cast<const T *>(nullptr));
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) qv[s][k] = fl_ld_q(a, b, A, k, V, uv);
        }
        sv[s] = smooth(a, b, A, (int)uv);
    }
    float gu[NLMAX][3];
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        const float u0 = __expf(e0[L]);
#pragma unroll
        for (int k = 0; k < 3; ++k) gu[L][k] = h[k] ? __expf(en[L][k]) - u0 : 0.f;
        if (CH && L >= a.nl) gu[L][0] = gu[L][1] = gu[L][2] = 0.f;
    }
    // slot pairs, stored as they are formed; with 16-bit state a slot pair
    // is a node pair (2P, 2P + 1) of one packed word (NI and ni are even)
#pragma unroll
    for (int s = 0; s < NS; s += 2) {
        float p[2][3];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            p[j][0] = p[j][1] = p[j][2] = 0.f;
            if (SL::valid(a, s + j)) {
                float G[3];
                if (SL::tail(s + j)) {
                    const int L = s + j - NI;
                    G[0] = gu[L][0], G[1] = gu[L][1], G[2] = gu[L][2];
                } else {
                    if constexpr (CH)
                        grad_U_chain<NLMAX>(s + j, gu, G);
                    else
                        grad_U<3, NLMAX, false>(a, s + j, gu, G);
                }
                flow_project<3>(a, qv[s + j], G, h, sv[s + j], p[j]);
            }
        }
        if (store) {
            if constexpr (kPacked<T>) {
                if (SL::valid(a, s)) {
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        fl_st_q2<T, EXACT>(a, b, SL::node(a, s), k, V, uv, p[0][k], p[1][k]);
                }
            } else {
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    if (SL::valid(a, s + j)) {
#pragma unroll
                        for (int k = 0; k < 3; ++k)
                            sto(fld_w<float>(a.q_out, (b * a.nn + SL::node(a, s + j)) * 3 + k, V), uv,
                                p[j][k]);
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) pr[s + j][k] = roundtrip(p[j][k], static_cast<const T *>(nullptr));
    }
}

template <int NLMAX, int NI, bool TAIL, bool EXACT, typename T, bool CH = false>
__global__ __launch_bounds__(GTHREADS) void k_flow_label(StepArgs a, FusedGeom g) {
    using SL = Slots<NLMAX, NI, TAIL, EXACT>;
    constexpr int NS = SL::N;
    // new flows' x and y components: [slot][component][row + 1][column + 1],
    // row 0 the halo row y0 - 1 and column 0 the halo column x0 - 1
    __shared__ float lq[NS][2][GY + 1][GX + 1];
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
    float pzb[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) pzb[s] = 0.f;
    if (own && zs > 0) {
        float e0[NLMAX], pr[SL::NP][3];
        flow_point<NLMAX, NI, TAIL, EXACT, T, CH>(a, b, xa, ya, zs - 1, false, e0, pr);
#pragma unroll
        for (int s = 0; s < NS; ++s) pzb[s] = pr[s][2];
    }

    for (int z = zs; z < ze; ++z) {
        float e0[NLMAX], pz[NS], dl[NLMAX];
        if (va) {
            float pr[SL::NP][3];
            flow_point<NLMAX, NI, TAIL, EXACT, T, CH>(a, b, xa, ya, z, own, e0, pr);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                lq[s][0][lr][lc] = pr[s][0];
                lq[s][1][lr][lc] = pr[s][1];
                pz[s] = pr[s][2];
            }
        }
        if (own) {
            const unsigned uv = (unsigned)((z * a.ny + ya) * a.nx + xa);
#pragma unroll
            for (int L = 0; L < NLMAX; ++L)
                dl[L] = ldf(fld<float>(a.D, b * a.nl + (EXACT || L < a.nl ? L : a.nl - 1), V), uv);
        }
        __syncthreads();
        // label step of iteration k + 1 (label_body's expressions and order:
        // the nodes in order, the internal ones first)
        if (own) {
            const unsigned uv = (unsigned)((z * a.ny + ya) * a.nx + xa);
            const bool bwd[2] = {xa > 0, ya > 0};
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                // div_from's sum in its order; the forward terms need no
                // select (a new flow's component is +0 where the voxel is
                // last on its axis) nor does q_z below the first plane (pzb
                // starts at +0)
                float dv = 0.f;
                dv += lq[s][0][lr][lc];
                dv -= bwd[0] ? lq[s][0][lr][lc - 1] : 0.f;
                dv += lq[s][1][lr][lc];
                dv -= bwd[1] ? lq[s][1][lr - 1][lc] : 0.f;
                dv += pz[s];
                dv -= pzb[s];
                if (SL::tail(s)) {
                    dl[s - NI] += dv;
                } else {
                    if constexpr (CH)
                        add_excess_chain<NLMAX>(dl, s, dv);
                    else
                        add_excess<NLMAX, false>(a, dl, s, dv);
                }
            }
            fl_entropic_step<NLMAX, EXACT>(a, dl, e0);
#pragma unroll
            for (int L = 0; L < NLMAX; L += 2) fl_st_ell2<T, EXACT>(a, b, L, V, uv, e0[L], e0[L + 1]);
#pragma unroll
            for (int s = 0; s < NS; ++s) pzb[s] = pz[s];
        }
        __syncthreads();   // the plane's LDS flows are read
    }
}

// ----------------------------------------------------------- dispatch ----

}  // namespace

bool flow_label_supported(int nd, int nl, int nn, bool identity) {
    return nd == 3 && !identity && nl <= 16 && nn <= 16;
}

// Builds with identity slots: at most 8 internal nodes (and 4 with more than
// 12 leaves), an even count of them with 16-bit state unless the graph fills
// an exact build (3 internal nodes over 8 leaves: the HMF tree).
bool flow_label_tail_supported(int nl, int nn, int storage) {
    const int ni = nn - nl;
    if (ni < 0 || ni > 8 || (ni > 4 && nl > 12)) return false;
    return storage == PF_FP32 || ni % 2 == 0 || (ni == 3 && nl == 8);
}

// Graphs whose end-labels are the last nodes and fill every slot of a build
// with identity slots (the EXACT forms: 4, 8, 12 or 16 leaves under 4
// internal nodes, 8 or 12 leaves under 8, 8 leaves under 3).
static bool flow_label_tail_exact(int nl, int nn) {
    const int ni = nn - nl;
    return (ni == 4 && nl % 4 == 0 && nl <= 16 && nn <= 16) || (ni == 8 && (nl == 8 || nl == 12) && nn <= 16) ||
           (ni == 3 && nl == 8);
}

// PF_KERNEL_AUTO takes this pass where it measured faster than the two-pass
// kernels on MI355X (per iteration at 128x256x256 unless stated, z chunks
// of 32 planes): every label graph with float32 state (DAGMF 256x512x512
// 8.68 against 10.6-11.5 ms, the HMF tree 0.720 against 0.836; random DAGs
// and trees of 3 to 16 flows 1.035-1.24x faster), and every storage type for
// the EXACT forms (DAGMF bf16 4.97-4.99 against 5.60 ms, fp16 4.97 against
// 5.73; the HMF tree bf16 0.436 against 0.483; random DAGs of 4/8, 8/8, 4/12
// and 4/4 internal nodes / leaves, bf16: 1.07-1.20x).  Otherwise, with
// 16-bit state, the two-pass kernels stay ahead (non-exact DAGs of 2/6 and
// 6/10: 0.84x and 0.79x): this pass issues more instructions than the two
// passes (halo recomputation, and the slot and label masks of graphs that
// do not fill the build) at one block per compute unit, while the two
// passes are bound by memory bandwidth.  The Ishikawa chain, the only graph
// with fewer flows than labels, runs builds of 4, 8, 12 or 16 labels with its
// weights fixed; it takes this pass with float32 state where it leaves at
// most 2 padding labels in its build (3, 4, 6, 8, 10, 12 and 16 labels:
// 1.46, 1.24, 1.05, 1.11, 1.14, 1.15 and 1.11x; 5 labels: 0.95x) and with
// 16-bit state up to 4 labels (bf16 1.31 and 1.07x; 8, 12 and 16 labels
// 1.00-1.02x, 5, 6 and 10 labels 0.78-0.95x).
bool flow_label_preferred(int nd, int nl, int nn, bool identity, int storage, bool tail) {
    if (!flow_label_supported(nd, nl, nn, identity)) return false;
    if (nn == nl - 1) {
        const int build = nl <= 4 ? 4 : nl <= 8 ? 8 : nl <= 12 ? 12 : 16;
        return storage == PF_FP32 ? build - nl <= 2 : nl <= 4;
    }
    if (tail && flow_label_tail_exact(nl, nn) && flow_label_tail_supported(nl, nn, storage)) return true;
    return storage == PF_FP32;
}

// z chunks of about 32 planes (each chunk recomputes one flow plane below
// it), but at least one block per compute unit, and chunks of at least 16
// planes.  Measured per iteration against chunk counts from 1 to 16: DAGMF
// 256x512x512 (512 tiles, 8 chunks) fp32 8.69 ms (9.30 with 1 or 2 chunks,
// 9.00 with 4), bf16 4.99-5.00 (5.00-5.02 with 1-4, 5.09 with 16); HMF
// 128x256x256 (128 tiles, 4 chunks) fp32 0.724 ms, bf16 0.466 (2 chunks:
// 0.71, 0.454; 8: 0.753, 0.473; 1 chunk leaves half the compute units idle).
FusedGeom flow_label_geometry(const StepArgs &a) {
    const long tiles = (long)((a.nx + GX - 1) / GX) * ((a.ny + GY - 1) / GY) * a.B;
    const long by_depth = tiles * ((a.nz + 31) / 32);
    return tile_geometry(a, GX, GY, by_depth > 256 ? by_depth : 256);
}

hipError_t launch_flow_label(const StepArgs &a, int storage, bool tail, hipStream_t s) {
    if (!flow_label_supported(3, a.nl, a.nn, false) || a.nz < 1) return hipErrorInvalidValue;
    const FusedGeom g = flow_label_geometry(a);
    if (g.blocks <= 0 || g.blocks > 0x7fffffffL) return hipErrorInvalidValue;
    const int ni = a.nn - a.nl;
    tail = tail && flow_label_tail_supported(a.nl, a.nn, storage);
    // tail builds also come in an EXACT form for graphs that fill every slot
    // (a tail build with an odd internal count exists only in the EXACT form)
    auto go = [&]<int NL, int NI, bool TL, typename T>() {
        if (TL && a.nl == NL && a.nn - a.nl == NI)
            k_flow_label<NL, NI, TL, TL, T><<<(unsigned)g.blocks, GTHREADS, 0, s>>>(a, g);
        else if constexpr (!(TL && NI % 2 == 1))
            k_flow_label<NL, NI, TL, false, T><<<(unsigned)g.blocks, GTHREADS, 0, s>>>(a, g);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    };
    // the Ishikawa chain, the only graph with fewer flows than labels, runs
    // the builds with its path weights fixed
    auto chain = [&]<int NL, typename T>() {
        k_flow_label<NL, NL, false, false, T, true><<<(unsigned)g.blocks, GTHREADS, 0, s>>>(a, g);
        return hipGetLastError();
    };
    auto by = [&]<typename T>() -> hipError_t {
        if (a.nn == a.nl - 1) {
            if (a.nl <= 4) return chain.template operator()<4, T>();
            if (a.nl <= 8) return chain.template operator()<8, T>();
            if (a.nl <= 12) return chain.template operator()<12, T>();
            return chain.template operator()<16, T>();
        }
        if (tail) {
            if (ni == 3 && a.nl == 8) return go.template operator()<8, 3, true, T>();
            if (ni <= 4 && a.nl <= 4) return go.template operator()<4, 4, true, T>();
            if (ni <= 4 && a.nl <= 8) return go.template operator()<8, 4, true, T>();
            if (ni <= 4 && a.nl <= 12) return go.template operator()<12, 4, true, T>();
            if (ni <= 4) return go.template operator()<16, 4, true, T>();
            if (a.nl <= 8) return go.template operator()<8, 8, true, T>();
            return go.template operator()<12, 8, true, T>();
        }
        if (a.nl <= 4 && a.nn <= 8) return go.template operator()<4, 8, false, T>();
        if (a.nl <= 8 && a.nn <= 8) return go.template operator()<8, 8, false, T>();
        if (a.nl <= 8 && a.nn <= 12) return go.template operator()<8, 12, false, T>();
        if (a.nl <= 8 && a.nn <= 16) return go.template operator()<8, 16, false, T>();
        if (a.nl <= 12 && a.nn <= 16) return go.template operator()<12, 16, false, T>();
        return go.template operator()<16, 16, false, T>();
    };
    if (storage == PF_BF16) return by.template operator()<bf16s>();
    if (storage == PF_FP16) return by.template operator()<f16s>();
    return by.template operator()<float>();
}

}  // namespace pf
