// CPU launchers for the threaded build of the library's kernels: every block
// of a launch runs in turn; kernels that synchronise (LDS exchange, block
// reductions) run one OS thread per GPU thread with std::barrier standing in
// for __syncthreads.  The launch geometries and template buckets mirror the
// library's launchers.
#include "kernels.inc"
#include "fused.inc"
#include "flowlabel.inc"
#include "adjoint.inc"
#include "fullflow.inc"
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>
thread_local dim3 blockIdx, threadIdx;
dim3 gridDim, blockDim;
thread_local std::barrier<> *emu_bar;
extern "C" float __expf(float x) throw() { return expf(x); }
extern "C" float __logf(float x) throw() { return logf(x); }
extern "C" {
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, int, hipStream_t) { std::memcpy(d, s, n); return 0; }
hipError_t hipStreamSynchronize(hipStream_t) { return 0; }
const char *hipGetErrorString(hipError_t) { return "cpu build"; }
}
namespace pf {
using namespace dev;
template <typename F> static void run_grid(dim3 g, unsigned nt, bool threads, F f) {
    gridDim = g;
    blockDim = dim3(nt);
    for (unsigned z = 0; z < g.z; ++z)
        for (unsigned y = 0; y < g.y; ++y)
            for (unsigned x = 0; x < g.x; ++x) {
                if (!threads) {
                    for (unsigned t = 0; t < nt; ++t) {
                        blockIdx = dim3(x, y, z);
                        threadIdx = dim3(t);
                        emu_bar = nullptr;
                        f();
                    }
                    continue;
                }
                std::barrier<> bar(nt);
                std::vector<std::thread> th;
                th.reserve(nt);
                for (unsigned t = 0; t < nt; ++t)
                    th.emplace_back([&, t, x, y, z] {
                        blockIdx = dim3(x, y, z);
                        threadIdx = dim3(t);
                        emu_bar = &bar;
                        f();
                    });
                for (auto &h : th) h.join();
            }
}
static unsigned sblocks(size_t n) { size_t b = (n + 255) / 256; return (unsigned)(b < 4096 ? (b ? b : 1) : 4096); }
static dim3 vgrid(const StepArgs &a) { return dim3((unsigned)((a.V + 255) / 256), (unsigned)a.B, 1); }
size_t storage_bytes(int storage) { return storage == PF_FP32 ? 4 : 2; }
template <int ND, typename T, typename F> static hipError_t bucket(bool ident, int nl, int nn, F &f) {
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
template <typename F> static hipError_t disp(int nd, int st, bool ident, int nl, int nn, F &&f) {
    if (nd == 2) {
        if (st == PF_BF16) return bucket<2, bf16s>(ident, nl, nn, f);
        if (st == PF_FP16) return bucket<2, f16s>(ident, nl, nn, f);
        return bucket<2, float>(ident, nl, nn, f);
    }
    if (st == PF_BF16) return bucket<3, bf16s>(ident, nl, nn, f);
    if (st == PF_FP16) return bucket<3, f16s>(ident, nl, nn, f);
    return bucket<3, float>(ident, nl, nn, f);
}
template <typename F> static hipError_t dtype(int st, F &&f) {
    if (st == PF_BF16) return f.template operator()<bf16s>();
    if (st == PF_FP16) return f.template operator()<f16s>();
    return f.template operator()<float>();
}
hipError_t launch_upload(const ConstBlock &c, float *dst, hipStream_t) {
    run_grid(dim3((kConstFloats + 255) / 256), 256, false, [&] { k_upload(c, dst); });
    return 0;
}
hipError_t launch_init(const StepArgs &a, int nd, int st, float ell0, hipStream_t) {
    size_t ne = (size_t)a.B * state_fields(a.nl, st) * a.V, nq = (size_t)a.B * state_fields(a.nn, st) * nd * a.V;
    return dtype(st, [&]<typename T>() {
        run_grid(dim3(sblocks(ne > nq ? ne : nq)), 256, false, [&] { k_init<T>((T *)a.ell_out, ne, (T *)a.q_out, nq, ell0); });
        return 0;
    });
}
hipError_t launch_copy_state(const StepArgs &a, int nd, int st, hipStream_t) {
    size_t ne = (size_t)a.B * state_fields(a.nl, st) * a.V, nq = (size_t)a.B * state_fields(a.nn, st) * nd * a.V;
    return dtype(st, [&]<typename T>() {
        run_grid(dim3(sblocks(nq)), 256, false, [&] {
            k_copy<T>((const T *)a.ell_in, (T *)a.ell_out, ne, (const T *)a.q_in, (T *)a.q_out, nq);
        });
        return 0;
    });
}
hipError_t launch_label(const StepArgs &a, bool ident, int nd, int st, hipStream_t) {
    return disp(nd, st, ident, a.nl, a.nn, [&]<int ND, int NL, int NN, bool ID, typename T>() {
        run_grid(vgrid(a), 256, false, [&] { k_label<ND, NL, NN, ID, T>(a); });
        return 0;
    });
}
hipError_t launch_flow(const StepArgs &a, bool ident, int nd, int st, hipStream_t) {
    return disp(nd, st, ident, a.nl, a.nn, [&]<int ND, int NL, int NN, bool ID, typename T>() {
        run_grid(vgrid(a), 256, false, [&] { k_flow<ND, NL, NN, ID, T>(a); });
        return 0;
    });
}
hipError_t launch_lds(const StepArgs &a, bool ident, int st, int iters, hipStream_t) {
    if (!lds_supported(2, a.nl, a.nn, a.V) || a.nz != 1 || iters < 1) return 1;
    return disp(2, st, ident, a.nl, a.nn, [&]<int ND, int NL, int NN, bool ID, typename T>() {
        run_grid(dim3((unsigned)a.B), kLdsThreads, true, [&] { k_lds2d<NL, NN, ID, T>(a, iters); });
        return 0;
    });
}
hipError_t launch_tile(const StepArgs &a, bool ident, int st, int iters, hipStream_t) {
    const TileGeom g = tile_geometry(a.nx, a.ny, a.B, a.nn);
    if (!tile_supported(2, a.nl, a.nn) || a.nz != 1 || iters < 1 || iters > g.k) return 1;
    const unsigned blocks = (unsigned)(g.tiles_x * g.tiles_y * a.B);
    return disp(2, st, ident, a.nl, a.nn, [&]<int ND, int NL, int NN, bool ID, typename T>() {
        if constexpr (NL <= 8 && NN <= 16) {
            if (g.rw * g.rh > tile_threads(NN)) return 1;
            run_grid(dim3(blocks), tile_threads(NN), true, [&] { k_tile2d<NL, NN, ID, T>(a, g, iters); });
            return 0;
        }
        return 1;
    });
}
hipError_t launch_fused(const StepArgs &a, bool ident, int nd, int st, hipStream_t) {
    const FusedGeom g = fused_geometry(a);
    auto f = [&]<int ND, int NL, int NN, bool ID, typename T>() {
        // the fused builds for label graphs: the two-pass buckets in 3-D,
        // (4, 8), (8, 16), (16, 16) in 2-D
        constexpr int NL2 = (ID || ND == 3) ? NL : (NL > 8 ? 16 : NL);
        constexpr int NN2 = (ID || ND == 3) ? NN : (NL2 == 4 ? 8 : 16);
        run_grid(dim3((unsigned)g.blocks), FTHREADS, true, [&] { k_fused<ND, NL2, NN2, ID, T>(a, g); });
        return 0;
    };
    return disp(nd, st, ident, a.nl, a.nn, f);
}
hipError_t launch_fused2(const StepArgs &a, int st, hipStream_t) {
    if (!fused2_supported(3, a.nl, a.nn, true) || a.nz < 1) return 1;
    const FusedGeom g = fused2_geometry(a);
    return dtype(st, [&]<typename T>() {
        if (a.nl <= 4) run_grid(dim3((unsigned)g.blocks), T2THREADS, true, [&] { k_fused2<4, T>(a, g); });
        else run_grid(dim3((unsigned)g.blocks), T2THREADS, true, [&] { k_fused2<8, T>(a, g); });
        return 0;
    });
}
hipError_t launch_flow_label(const StepArgs &a, int st, bool tail, hipStream_t) {
    if (!flow_label_supported(3, a.nl, a.nn, false) || a.nz < 1) return 1;
    const FusedGeom g = flow_label_geometry(a);
    const int ni = a.nn - a.nl;
    tail = tail && flow_label_tail_supported(a.nl, a.nn, st);
    auto go = [&]<int NL, int NI, bool TL, typename T>() {
        if (TL && a.nl == NL && a.nn - a.nl == NI)
            run_grid(dim3((unsigned)g.blocks), GTHREADS, true, [&] { k_flow_label<NL, NI, TL, TL, T>(a, g); });
        else if constexpr (!(TL && NI % 2 == 1))
            run_grid(dim3((unsigned)g.blocks), GTHREADS, true, [&] { k_flow_label<NL, NI, TL, false, T>(a, g); });
        else
            return 1;
        return 0;
    };
    auto chain = [&]<int NL, typename T>() {
        run_grid(dim3((unsigned)g.blocks), GTHREADS, true, [&] { k_flow_label<NL, NL, false, false, T, true>(a, g); });
        return 0;
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
    return dtype(st, by);
}
hipError_t launch_energy(const StepArgs &a, bool ident, int nd, int st, double *partials, double *results,
                         hipStream_t) {
    // fewer blocks than the library (64, not kPartials) keep the threaded run
    // short; the unused partials are set to the reduction's neutral values
    hipError_t e = disp(nd, st, ident, a.nl, a.nn, [&]<int ND, int NL, int NN, bool ID, typename T>() {
        run_grid(dim3(64), 256, true, [&] { k_energy<ND, NL, NN, ID, T>(a, partials); });
        return 0;
    });
    for (int i = 64 * 4; i < kPartials * 4; ++i) partials[i] = (i % 4 == 3) ? -INFINITY : 0.0;
    run_grid(dim3(1), 256, true, [&] { k_reduce(partials, kPartials, results); });
    return e;
}
hipError_t launch_export(const StepArgs &a, int nd, int st, float *u, int32_t *labels, float *q, hipStream_t) {
    return dtype(st, [&]<typename T>() {
        if (nd == 2) run_grid(vgrid(a), 256, false, [&] { k_export<2, T>(a, u, labels, q); });
        else run_grid(vgrid(a), 256, false, [&] { k_export<3, T>(a, u, labels, q); });
        return 0;
    });
}
hipError_t launch_export_ell(const StepArgs &a, int st, float *ell, hipStream_t) {
    return dtype(st, [&]<typename T>() {
        run_grid(vgrid(a), 256, false, [&] { k_export_ell<T>(a, ell); });
        return 0;
    });
}
hipError_t launch_check(const StepArgs &, int32_t *, hipStream_t) { std::abort(); }
template <typename F> static hipError_t adisp(int nd, bool ident, int nl, int nn, F &&f) {
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
hipError_t launch_adj_flow(const StepArgs &a, const AdjArgs &g, bool ident, int nd, hipStream_t) {
    return adisp(nd, ident, a.nl, a.nn, [&]<int ND, int NL, int NN, bool ID>() {
        run_grid(vgrid(a), 256, false, [&] { k_adj_flow<ND, NL, NN, ID>(a, g); });
        return 0;
    });
}
hipError_t launch_adj_label(const StepArgs &a, const AdjArgs &g, bool ident, int nd, hipStream_t) {
    return adisp(nd, ident, a.nl, a.nn, [&]<int ND, int NL, int NN, bool ID>() {
        run_grid(vgrid(a), 256, false, [&] { k_adj_label<ND, NL, NN, ID>(a, g); });
        return 0;
    });
}
hipError_t launch_adj_fused(const StepArgs &a, const AdjArgs &g, bool ident, int nd, hipStream_t) {
    if (!adj_fused_supported(nd, a.nl, a.nn, ident)) return 1;
    const FusedGeom geo = tile_geometry(a, RTX, RTY);
    // 2-D rows of up to ROW_COLS voxels: the row march, same chunking as the library
    const bool rows = nd == 2 && a.nx <= ROW_COLS;
    const long waves = (long)a.B * ((a.nx + 63) / 64);
    const long want = (4096 + waves - 1) / waves, max_chunks = (a.ny + 3) / 4;
    const int n0 = (int)(want < max_chunks ? want : max_chunks);
    const int cy = (a.ny + n0 - 1) / n0, n_chunks = (a.ny + cy - 1) / cy;
    auto f = [&]<int ND, int NL, int NN, bool ID>() {
        if constexpr (ND == 2) {
            if (rows) {
                run_grid(dim3((unsigned)(a.B * n_chunks)), (unsigned)((a.nx + 63) / 64 * 64), true,
                         [&] { k_adj_rows<NL, NN, ID>(a, g, cy, n_chunks); });
                return 0;
            }
        }
        run_grid(dim3((unsigned)geo.blocks), RTHREADS, true, [&] { k_adj_fused<ND, NL, NN, ID>(a, g, geo); });
        return 0;
    };
    if (nd == 2) {
        if (!ident) return f.template operator()<2, 4, 8, false>();
        if (a.nl <= 4) return f.template operator()<2, 4, 4, true>();
        if (a.nl <= 6) return f.template operator()<2, 6, 6, true>();
        return f.template operator()<2, 8, 8, true>();
    }
    return f.template operator()<3, 4, 4, true>();
}
hipError_t launch_fill(float *p, size_t n, float val, hipStream_t) {
    if (n) run_grid(dim3(sblocks(n)), 256, false, [&] { k_fill(p, n, val); });
    return 0;
}
hipError_t launch_copy_f(const float *x, float *y, size_t n, hipStream_t) {
    if (n) run_grid(dim3(sblocks(n)), 256, false, [&] { k_copy_f(x, y, n); });
    return 0;
}
hipError_t launch_sum_nodes(const float *sbar, int B, int nn, size_t V, float *out, hipStream_t) {
    run_grid(dim3(nn), 256, true, [&] { k_sum_nodes(sbar, B, nn, V, out); });
    return 0;
}
template <typename F> static hipError_t ffdisp(int nd, int n, F &&f) {
    auto by = [&]<int ND>() -> hipError_t {
        if (n <= 4) return f.template operator()<ND, 4>();
        if (n <= 8) return f.template operator()<ND, 8>();
        return f.template operator()<ND, 16>();
    };
    return nd == 2 ? by.template operator()<2>() : by.template operator()<3>();
}
hipError_t launch_ff_init(const StepArgs &a, const FFArgs &f, int nd, hipStream_t) {
    return ffdisp(nd, a.nl, [&]<int ND, int NL>() {
        run_grid(vgrid(a), kBlock, false, [&] { k_ff_init<ND, NL>(a, f); });
        return 0;
    });
}
hipError_t launch_ff_iteration(const StepArgs &a, const FFArgs &f, int nd, hipStream_t) {
    return ffdisp(nd, a.nl, [&]<int ND, int NL>() {
        run_grid(vgrid(a), kBlock, false, [&] { k_ff_flow<ND, NL>(a, f); });
        run_grid(vgrid(a), kBlock, false, [&] { k_ff_rest<ND, NL>(a, f); });
        return 0;
    });
}
hipError_t launch_ff_energy(const StepArgs &a, const FFArgs &f, int nd, double *partials, double *results,
                            hipStream_t) {
    // 64 blocks, not kPartials, as launch_energy above
    hipError_t e = ffdisp(nd, a.nl, [&]<int ND, int NL>() {
        run_grid(dim3(64), kBlock, true, [&] { k_ff_energy<ND, NL>(a, f, partials); });
        return 0;
    });
    for (int i = 64 * 4; i < kPartials * 4; ++i) partials[i] = (i % 4 == 3) ? -INFINITY : 0.0;
    run_grid(dim3(1), kBlock, true, [&] { k_ff_reduce(partials, kPartials, results); });
    return e;
}
hipError_t launch_ff_export(const StepArgs &a, const FFArgs &f, int nd, float *u, int32_t *labels, float *q,
                            hipStream_t) {
    return ffdisp(nd, a.nl, [&]<int ND, int NL>() {
        run_grid(vgrid(a), kBlock, false, [&] { k_ff_export<ND, NL>(a, f, u, labels, q); });
        return 0;
    });
}
}  // namespace pf
