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
// flow one plane below (ignored at z == 0).  Returns the new log-labels as
// stored (er: after the round trip through the storage type, what a later
// load returns), the new labels u = exp(er) (what the two-pass flow kernel
// reads back), the old flows at the voxel in qpt, and stores the new
// log-labels when `store`.  All loads are issued first, unconditionally.
template <int ND, int NLMAX, int NNMAX, bool IDENT, typename T, bool N32 = false>
__device__ __forceinline__ void label_point(const StepArgs &a, int b, int x, int y, int z,
                                            const float (&qzb)[NNMAX], bool store,
                                            float (&u)[NLMAX], float (&qpt)[NNMAX][ND],
                                            float (&er)[NLMAX]) {
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
        d[L] = ldf(field<float, N32>(a.D, b, a.nl, Lc, V), uv);
        e[L] = ld_ell<T, N32>(a.ell_in, b, a.nl, L, V, uv);
    }
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) {
        qpt[A][0] = ld_q<T, ND, N32>(a.q_in, b, a.nn, A, 0, V, uv);
        qpt[A][1] = ld_q<T, ND, N32>(a.q_in, b, a.nn, A, 1, V, uv);
        if constexpr (ND == 3) qpt[A][2] = ld_q<T, ND, N32>(a.q_in, b, a.nn, A, 2, V, uv);
        qm[A][0] = ld_q<T, ND, N32>(a.q_in, b, a.nn, A, 0, V, uv - (unsigned)m[0]);
        qm[A][1] = ld_q<T, ND, N32>(a.q_in, b, a.nn, A, 1, V, uv - (unsigned)m[1]);
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
        for (int L = 0; L < NLMAX; L += 2) st_ell2<T, N32>(a.ell_out, b, a.nl, L, V, uv, e[L], e[L + 1]);
    }
#pragma unroll
    for (int L = 0; L < NLMAX; ++L) {
        er[L] = roundtrip(e[L], static_cast<const T *>(nullptr));
        u[L] = __expf(er[L]);
    }
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

    // Each thread has one point: rows 0 .. FTY-1 an owned voxel column, row
    // FTY the halo row past the tile, row FTY+1 (its own wavefronts) the
    // column past the tile.  One set of carried registers serves either kind.
    const bool colp = row == FTY + 1;
    const int xa = colp ? x0 + FTX : x0 + col;
    const int ya = colp ? y0 + col : y0 + row;
    const bool va = (colp ? col < FTY : row <= FTY) && xa < a.nx && ya < a.ny;
    const bool own = row < FTY && va;
    const int lr = colp ? col : row, lc = colp ? FTX : col;   // LDS slot of the point

    const size_t V = (size_t)a.V;

    float ua[NLMAX], er[NLMAX];   // er: unused here
    float qa[NNMAX][ND];
    float qzb[NNMAX];
#pragma unroll
    for (int A = 0; A < NNMAX; ++A) qzb[A] = 0.f;

    // prologue: labels of plane zs, old q_z of plane zs - 1
    if (va) {
        if (ND == 3 && zs > 0) {
            const int vbelow = ((zs - 1) * a.ny + ya) * a.nx + xa;
#pragma unroll
            for (int A = 0; A < NNMAX; ++A)
                qzb[A] = ld_q<T, ND>(a.q_in, b, a.nn, A, ND - 1, V, (unsigned)vbelow);
        }
        label_point<ND, NLMAX, NNMAX, IDENT, T>(a, b, xa, ya, zs, qzb, own, ua, qa, er);
#pragma unroll
        for (int L = 0; L < NLMAX; ++L) lds[L][lr][lc] = ua[L];
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
        float un[NLMAX], qn[NNMAX][ND];
#pragma unroll
        for (int L = 0; L < NLMAX; ++L) un[L] = ua[L];   // defined when !has_next
        // labels of plane z + 1 (owned when z + 1 < ze, else the halo plane)
        if (va && has_next) {
            float qz[NNMAX];
#pragma unroll
            for (int A = 0; A < NNMAX; ++A) qz[A] = qa[A][ND - 1];
            label_point<ND, NLMAX, NNMAX, IDENT, T>(a, b, xa, ya, z + 1, qz, own && z + 1 < ze,
                                                    un, qn, er);
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
        if (has_next && va) {
#pragma unroll
            for (int L = 0; L < NLMAX; ++L) {
                lds[L][lr][lc] = un[L];
                ua[L] = un[L];
            }
#pragma unroll
            for (int A = 0; A < NNMAX; ++A)
#pragma unroll
                for (int k = 0; k < ND; ++k) qa[A][k] = qn[A][k];
        }
        __syncthreads();
    }
}

// ------------------------------------------------ two iterations per pass ----
// Temporal blocking for 3-D Potts: iterations k -> k+1 -> k+2 in one z-march,
// so that the state is read and written once per two iterations.  The
// dependency cone of the owned tile [x0, x0+TW) x [y0, y0+TH) widens by one
// voxel per step in x and y:
//   second flow step   on the owned tile           (stage D)
//   second label step  on [x0, x0+TW] x [y0, y0+TH]   (forward neighbours, C)
//   first flow step    on [x0-1, x0+TW] x [y0-1, y0+TH] (backward neighbours
//                      of the divergence, B)
//   first label step   on [x0-1, x0+TW+1] x [y0-1, y0+TH+1]   (A)
// One thread per column of the widest region (RW x RH); along z the stages
// lag, so that at step z the block computes A on plane z+2, B and C on plane
// z+1 and D on plane z.  Per column a thread carries in registers the old
// flows of plane z+1 (for B, and as the z-neighbour of A), the first
// iteration's log-labels of plane z+1 (for C) and its flows of plane z (for
// D, and as the z-neighbour of C); the x/y neighbours go through LDS (the
// first iteration's labels for B, its x/y flow components for C, the second
// iteration's labels for D).  Intermediate values are rounded to the storage
// type exactly where the single-iteration kernels store and reload them, and
// every point uses the same expressions, so the result equals two fused (or
// two-pass) iterations bit for bit.
constexpr int TW = 64;                        // owned tile width
constexpr int TH = 8;                         // owned tile rows
constexpr int RW = TW + 3;                    // first label step's columns
constexpr int RH = TH + 3;                    // and rows
constexpr int T2THREADS = (RW * RH + 63) / 64 * 64;

template <int NL, typename T>
__global__ __launch_bounds__(T2THREADS) void k_fused2(StepArgs a, FusedGeom g) {
    constexpr int NN = NL;   // Potts: one flow per label
    __shared__ float lu1[NL][RH][RW];      // first-iteration labels, plane z+1
    __shared__ float lu2[NL][RH][RW];      // second-iteration labels, plane z
    __shared__ float lq1[NN][2][RH][RW];   // first-iteration q_x, q_y, plane z+1
    const int tid = threadIdx.x;
    const int r = tid / RW, c = tid % RW;

    // XCD-aware block -> tile mapping (as in k_fused)
    const int nb = gridDim.x;
    const int pb = blockIdx.x;
    const int lb = (nb % 8 == 0) ? (pb % 8) * (nb / 8) + pb / 8 : pb;
    const int bx = lb % g.tiles_x;
    int rr = lb / g.tiles_x;
    const int by = rr % g.tiles_y;
    rr /= g.tiles_y;
    const int ch = rr % g.n_chunks;
    const int b = rr / g.n_chunks;
    const int zs = ch * g.cz;
    const int ze = min(a.nz, zs + g.cz);

    const int x = bx * TW - 1 + c, y = by * TH - 1 + r;
    const bool inA = r < RH && x >= 0 && x < a.nx && y >= 0 && y < a.ny;
    const bool inB = inA && c <= TW + 1 && r <= TH + 1;
    const bool inC = inB && c >= 1 && r >= 1;
    const bool own = inC && c <= TW && r <= TH;
    const size_t V = (size_t)a.V;
    const float *Tn = nullptr;
    auto vox = [&](int p) { return (unsigned)((p * a.ny + y) * a.nx + x); };

    // carried: old flows of plane z+1, first-iteration log-labels of plane
    // z+1 and flows of plane z, data term of plane z+1, capacities of plane z
    float q0c[NN][3], e1c[NL], q1c[NN][3], dc[NL], sc[NN];
#pragma unroll
    for (int A = 0; A < NN; ++A) {
        e1c[A] = dc[A] = sc[A] = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) q0c[A][k] = q1c[A][k] = 0.f;
    }
    // first label step on plane zs - 1 (the first flow step there feeds the
    // z-neighbour of the second label step on plane zs)
    if (zs >= 1 && inA) {
        float qzb[NN], u[NL], er[NL];
#pragma unroll
        for (int A = 0; A < NN; ++A)
            qzb[A] = zs >= 2 ? ld_q<T, 3, true>(a.q_in, b, a.nn, A, 2, V, vox(zs - 2)) : 0.f;
        label_point<3, NL, NN, true, T, true>(a, b, x, y, zs - 1, qzb, false, u, q0c, er);
#pragma unroll
        for (int L = 0; L < NL; ++L) lu1[L][r][c] = u[L];
    }
    __syncthreads();

    for (int z = zs - 2; z < ze; ++z) {
        const int pA = z + 2, pB = z + 1;
        const bool doA = inA && pA < a.nz;
        const bool doB = inB && pB >= 0 && pB >= zs - 1 && pB < a.nz;
        const bool doC = inC && pB >= zs && pB < a.nz;
        const bool doD = own && z >= zs;

        // all global loads of the step are issued here: the first label
        // step's inputs (its data term is kept for the second label step one
        // step later) and the capacities of plane z + 1 (kept for the second
        // flow step one step later)
        float e1n[NL], u1n[NL], q0n[NN][3], dn[NL], sn[NN];
#pragma unroll
        for (int A = 0; A < NN; ++A) {
            e1n[A] = u1n[A] = dn[A] = sn[A] = 0.f;
#pragma unroll
            for (int k = 0; k < 3; ++k) q0n[A][k] = 0.f;
        }
        if (doB) {
#pragma unroll
            for (int A = 0; A < NN; ++A) sn[A] = smooth(a, b, A < a.nn ? A : a.nn - 1, (int)vox(pB));
        }
        // A: first label step, plane z + 2
        if (doA) {
#pragma unroll
            for (int L = 0; L < NL; ++L)
                dn[L] = ldf(field<float, true>(a.D, b, a.nl, L < a.nl ? L : a.nl - 1, V), vox(pA));
            float qzb[NN];
#pragma unroll
            for (int A = 0; A < NN; ++A) qzb[A] = q0c[A][2];
            label_point<3, NL, NN, true, T, true>(a, b, x, y, pA, qzb, false, u1n, q0n, e1n);
        }

        // B: first flow step, plane z + 1
        float q1n[NN][3];
#pragma unroll
        for (int A = 0; A < NN; ++A)
#pragma unroll
            for (int k = 0; k < 3; ++k) q1n[A][k] = 0.f;
        if (doB) {
            const bool h[3] = {x < a.nx - 1, y < a.ny - 1, pB + 1 < a.nz};
#pragma unroll
            for (int A = 0; A < NN; ++A) {
                if (A < a.nn) {
                    const float uo = lu1[A][r][c];
                    float gu[NL][3];
                    gu[A][0] = h[0] ? lu1[A][r][c + 1] - uo : 0.f;
                    gu[A][1] = h[1] ? lu1[A][r + 1][c] - uo : 0.f;
                    gu[A][2] = h[2] ? u1n[A] - uo : 0.f;
                    float G[3], p[3];
                    grad_U<3, NL, true>(a, A, gu, G);
                    flow_project<3>(a, q0c[A], G, h, sn[A], p);
#pragma unroll
                    for (int k = 0; k < 3; ++k) q1n[A][k] = roundtrip(p[k], (const T *)Tn);
                }
                lq1[A][0][r][c] = q1n[A][0];
                lq1[A][1][r][c] = q1n[A][1];
            }
        }
        __syncthreads();   // B's reads of lu1 are done, lq1 is written
        if (doA) {
#pragma unroll
            for (int L = 0; L < NL; ++L) lu1[L][r][c] = u1n[L];
        }

        // C: second label step, plane z + 1
        float u2n[NL];
#pragma unroll
        for (int L = 0; L < NL; ++L) u2n[L] = 0.f;
        if (doC) {
            const unsigned uv = vox(pB);
            const Coord cc{x, y, pB};
            int m[3];
            bool bwd[3];
            backward_offsets(cc, a, m, bwd);
            const bool fwd[3] = {x < a.nx - 1, y < a.ny - 1, pB < a.nz - 1};
            float d[NL], e[NL];
#pragma unroll
            for (int L = 0; L < NL; ++L) {
                d[L] = dc[L];
                e[L] = e1c[L];
            }
#pragma unroll
            for (int A = 0; A < NN; ++A) {
                const float q0[3] = {q1n[A][0], q1n[A][1], q1n[A][2]};
                const float qm[3] = {lq1[A][0][r][c - 1], lq1[A][1][r - 1][c], q1c[A][2]};
                add_excess<NL, true>(a, d, A, div_from<3>(q0, qm, fwd, bwd));
            }
            entropic_step<NL>(a, d, e);
            if (own && pB < ze) {
#pragma unroll
                for (int L = 0; L < NL; L += 2) st_ell2<T, true>(a.ell_out, b, a.nl, L, V, uv, e[L], e[L + 1]);
            }
#pragma unroll
            for (int L = 0; L < NL; ++L) u2n[L] = __expf(roundtrip(e[L], (const T *)Tn));
        }

        // D: second flow step, plane z (owned voxels)
        if (doD) {
            const unsigned v = vox(z);
            const bool h[3] = {x < a.nx - 1, y < a.ny - 1, z + 1 < a.nz};
#pragma unroll
            for (int A = 0; A < NN; A += 2) {
                if (A < a.nn) {
                    float p[2][3];
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const int Aj = A + j;
#pragma unroll
                        for (int k = 0; k < 3; ++k) p[j][k] = 0.f;
                        if (Aj < a.nn) {
                            const float uo = lu2[Aj][r][c];
                            float gu[NL][3];
                            gu[Aj][0] = h[0] ? lu2[Aj][r][c + 1] - uo : 0.f;
                            gu[Aj][1] = h[1] ? lu2[Aj][r + 1][c] - uo : 0.f;
                            gu[Aj][2] = h[2] ? u2n[Aj] - uo : 0.f;
                            float G[3];
                            grad_U<3, NL, true>(a, Aj, gu, G);
                            flow_project<3>(a, q1c[Aj], G, h, sc[Aj], p[j]);
                        }
                    }
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        st_q2<T, 3, true>(a.q_out, b, a.nn, A, k, V, v, p[0][k], p[1][k]);
                }
            }
        }
        __syncthreads();   // C's reads of lq1 and D's reads of lu2 are done
        if (doC) {
#pragma unroll
            for (int L = 0; L < NL; ++L) lu2[L][r][c] = u2n[L];
        }
#pragma unroll
        for (int A = 0; A < NN; ++A) {
            e1c[A] = e1n[A];
            dc[A] = dn[A];
            sc[A] = sn[A];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                q0c[A][k] = q0n[A][k];
                q1c[A][k] = q1n[A][k];
            }
        }
    }
}

template <int ND, typename T, typename F>
hipError_t fused_bucket(bool ident, int nl, int nn, F &f) {
    if (ident) {
        if (nl <= 4) return f.template operator()<ND, 4, 4, true, T>();
        if (nl <= 8) return f.template operator()<ND, 8, 8, true, T>();
        return f.template operator()<ND, 16, 16, true, T>();
    }
    // label graphs: the 3-D buckets of the two-pass kernels (up to 16 flows)
    if (nl <= 4 && nn <= 8) return f.template operator()<ND, 4, 8, false, T>();
    if constexpr (ND == 3) {
        if (nl <= 8 && nn <= 8) return f.template operator()<ND, 8, 8, false, T>();
        if (nl <= 8 && nn <= 12) return f.template operator()<ND, 8, 12, false, T>();
    }
    if (nl <= 8 && nn <= 16) return f.template operator()<ND, 8, 16, false, T>();
    if constexpr (ND == 3) {
        if (nl <= 12 && nn <= 16) return f.template operator()<ND, 12, 16, false, T>();
    }
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
// two-pass kernels on MI355X (3-D Potts with float32 state; up to 8 labels
// the two-iteration pass below is faster still); the two-pass kernels
// elsewhere (their lower register pressure wins for 16-bit state and for
// label graphs).
bool fused_preferred(int nd, int nl, int nn, bool identity, int storage) {
    return identity && nd == 3 && storage == PF_FP32 && fused_supported(nd, nl, nn, identity);
}

FusedGeom fused_geometry(const StepArgs &a) { return tile_geometry(a, FTX, FTY); }

bool fused2_supported(int nd, int nl, int nn, bool identity) {
    return nd == 3 && identity && nl <= 8 && nn == nl;
}

// PF_KERNEL_AUTO takes two iterations per pass for 3-D Potts up to 8 labels,
// in every storage type: measured faster than the one-iteration pass and
// than the two-pass kernels at 256^3 (fp32 0.87 against 1.19 and 1.35 ms per
// iteration; bf16 0.68 against 0.82 and 0.72; fp16 0.64 against 0.72).
bool fused2_preferred(int nd, int nl, int nn, bool identity, int storage) {
    (void)storage;
    return fused2_supported(nd, nl, nn, identity);
}

// One block per compute unit (its register and LDS use allow no second one):
// about 256 blocks, i.e. few long z chunks; each chunk recomputes about three
// planes of the first iteration.
FusedGeom fused2_geometry(const StepArgs &a) { return tile_geometry(a, TW, TH, 256); }

FusedGeom tile_geometry(const StepArgs &a, int width, int rows, long target) {
    FusedGeom g{};
    g.tiles_x = (a.nx + width - 1) / width;
    g.tiles_y = (a.ny + rows - 1) / rows;
    const long tiles = (long)g.tiles_x * g.tiles_y * a.B;
    // by default about two resident blocks per compute unit on 256 CUs, with
    // chunks of at least 16 planes (each chunk recomputes one extra plane)
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

hipError_t launch_fused2(const StepArgs &a, int storage, hipStream_t s) {
    if (!fused2_supported(3, a.nl, a.nn, true) || a.nz < 1) return hipErrorInvalidValue;
    const FusedGeom g = fused2_geometry(a);
    if (g.blocks <= 0 || g.blocks > 0x7fffffffL) return hipErrorInvalidValue;
    auto go = [&]<int NL, typename T>() {
        k_fused2<NL, T><<<(unsigned)g.blocks, T2THREADS, 0, s>>>(a, g);
        return hipGetLastError();
    };
    auto by = [&]<typename T>() {
        return a.nl <= 4 ? go.template operator()<4, T>() : go.template operator()<8, T>();
    };
    if (storage == PF_BF16) return by.template operator()<bf16s>();
    if (storage == PF_FP16) return by.template operator()<f16s>();
    return by.template operator()<float>();
}

}  // namespace pf
