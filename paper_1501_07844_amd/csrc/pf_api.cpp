// Host side of the C ABI declared in pseudoflow.h: argument and label-graph
// validation, path-weight packing, workspace layout, the iteration loop with
// optional gap evaluations, export and timing.  All device work is enqueued
// through the launchers of pf_kernels.hip; nothing here allocates device
// memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pf_fullflow.h"
#include "pf_internal.h"
#include "pseudoflow.h"

namespace pf {

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Layout make_layout(const pf_grid &g, int nl, int nn, int storage, bool pingpong) {
    Layout L{};
    const size_t V = (size_t)g.nx * g.ny * g.nz;
    const size_t s = storage_bytes(storage);
    size_t off = 0;
    L.results = off;
    off += 256;
    L.flags = off;
    off += 256;
    L.consts = off;
    off = align256(off + sizeof(ConstBlock));
    L.partials = off;
    off = align256(off + (size_t)kPartials * 4 * sizeof(double));
    const size_t ell_b = align256((size_t)g.batch * state_fields(nl, storage) * V * s);
    const size_t q_b = align256((size_t)g.batch * state_fields(nn, storage) * g.ndim * V * s);
    L.ell[0] = off;
    off += ell_b;
    L.q[0] = off;
    off += q_b;
    if (pingpong) {
        L.ell[1] = off;
        off += ell_b;
        L.q[1] = off;
        off += q_b;
    } else {
        L.ell[1] = L.ell[0];
        L.q[1] = L.q[0];
    }
    L.total = off;
    return L;
}

}  // namespace pf

using namespace pf;

// Device scratch of solve_dagmf_static (callers that cannot allocate device
// memory): every GPU the library runs on holds one copy until the process
// ends.  Host code never passes this name to a kernel or a copy: it stands
// for a host-side shadow; the device address of each GPU's copy comes from
// hipGetSymbolAddress with that GPU current (static_scratch below).
static __device__ __align__(256) unsigned char scratch[PF_STATIC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(PF_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// A validated problem, ready to launch.
struct Prob {
    pf_grid g{};
    int nl = 0, nn = 0;
    const float *D = nullptr;
    const float *S = nullptr;
    int s_mode = 0;
    bool ident = true;
    bool tail = false;       // the last nl nodes are the end-labels, in order
    GraphW w{};
    float s_node[PF_MAX_NODES] = {};
};

int check_grid(const pf_grid *g) {
    if (!g) return fail(PF_EINVAL, "grid is NULL");
    if (g->ndim != 2 && g->ndim != 3) return fail(PF_EINVAL, "ndim must be 2 or 3 (got %d)", g->ndim);
    if (g->batch < 1 || g->nx < 1 || g->ny < 1 || g->nz < 1)
        return fail(PF_EINVAL, "grid extents must be >= 1 (batch %d, %d x %d x %d)", g->batch,
                    g->nz, g->ny, g->nx);
    if (g->ndim == 2 && g->nz != 1) return fail(PF_EINVAL, "ndim == 2 requires nz == 1 (got %d)", g->nz);
    if (g->batch > 65535) return fail(PF_EUNSUPPORTED, "batch > 65535");
    // byte offsets of 4-byte fields inside one problem stay below 2^32
    const double V = (double)g->nx * g->ny * g->nz;
    if (V > 1073741824.0 - 2.0 * g->nx * g->ny)
        return fail(PF_EUNSUPPORTED, "more than 2^30 voxels per problem");
    return PF_OK;
}

int check_inputs_common(Prob &p, const float *D, const float *S, int s_mode) {
    if (!D) return fail(PF_EINVAL, "D is NULL");
    if (!aligned(D, 4)) return fail(PF_EINVAL, "D is not 4-byte aligned");
    if (s_mode < PF_S_NODE_SCALAR || s_mode > PF_S_NODE_FIELD)
        return fail(PF_EINVAL, "unknown s_mode %d", s_mode);
    if (!S) return fail(PF_EINVAL, "S is NULL");
    p.D = D;
    p.s_mode = s_mode;
    if (s_mode == PF_S_NODE_SCALAR) {
        for (int A = 0; A < p.nn; ++A) {
            const float s = S[A];
            if (!std::isfinite(s)) return fail(PF_ENONFINITE, "S[%d] is not finite", A);
            if (s < 0.f) return fail(PF_EINVAL, "S[%d] = %g is negative", A, (double)s);
            p.s_node[A] = s;
        }
        p.S = nullptr;
    } else {
        if (!aligned(S, 4)) return fail(PF_EINVAL, "S is not 4-byte aligned");
        p.S = S;
    }
    return PF_OK;
}

// Device address of the static scratch on the current device, looked up
// once per device (with that device current) and kept.  The stream, if
// given, must belong to the current device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int static_scratch(hipStream_t stream, void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (stream) {
        hipDevice_t sdev = -1;
        if ((e = hipStreamGetDevice(stream, &sdev)) != hipSuccess) return hip_fail(e, "hipStreamGetDevice");
        if (sdev != dev)
            return fail(PF_EINVAL, "the stream belongs to device %d, the current device is %d", (int)sdev, dev);
    }
    if (dev < 0 || dev >= kMaxDevices)
        return fail(PF_EUNSUPPORTED, "device ordinal %d outside 0..%d", dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess)
            return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(PF_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PF_OK;
}

int check_params(const pf_params *P, bool static_ws = false) {
    if (!P) return fail(PF_EINVAL, "params is NULL");
    if (P->iters < 0) return fail(PF_EINVAL, "iters must be >= 0 (got %d)", P->iters);
    if (!(P->c > 0.f) || !std::isfinite(P->c)) return fail(PF_EINVAL, "c must be finite and > 0");
    if (!(P->tau > 0.f) || !std::isfinite(P->tau))
        return fail(PF_EINVAL, "tau must be finite and > 0");
    if (P->storage < PF_FP32 || P->storage > PF_FP16)
        return fail(PF_EINVAL, "unknown storage %d", P->storage);
    if (P->kernel < PF_KERNEL_AUTO || P->kernel > PF_KERNEL_LDS)
        return fail(PF_EINVAL, "unknown kernel %d", P->kernel);
    if (P->gap_every < 0) return fail(PF_EINVAL, "gap_every must be >= 0");
    if (!(P->gap_tol >= 0.0)) return fail(PF_EINVAL, "gap_tol must be >= 0");
    if (P->timing_stride < 0) return fail(PF_EINVAL, "timing_stride must be >= 0");
    if (static_ws) {
        if (P->workspace || P->workspace_bytes)
            return fail(PF_EINVAL, "the static-scratch solve takes no workspace "
                                   "(workspace must be NULL and workspace_bytes 0)");
        if (P->tape) return fail(PF_EUNSUPPORTED, "the static-scratch solve records no tape");
        if (P->timing_stride)
            return fail(PF_EUNSUPPORTED, "the static-scratch solve times no launches (timing_stride 0)");
        return PF_OK;
    }
    if (!P->workspace) return fail(PF_EINVAL, "workspace is NULL");
    if (!aligned(P->workspace, 256)) return fail(PF_EINVAL, "workspace is not 256-byte aligned");
    return PF_OK;
}

// Label graph -> path weights W[A][L]; checks acyclicity, reachability,
// weights and the unit source-to-leaf path sums.
int build_graph(const pf_graph *G, bool tree_only, Prob &p) {
    if (!G) return fail(PF_EINVAL, "graph is NULL");
    const int n = G->n_nodes, m = G->n_edges;
    if (n < 2) return fail(PF_EGRAPH, "graph needs a source and at least one label (n_nodes=%d)", n);
    if (n - 1 > PF_MAX_NODES)
        return fail(PF_EUNSUPPORTED, "%d non-source nodes > %d", n - 1, PF_MAX_NODES);
    if (m < 1 || !G->parent || !G->child) return fail(PF_EGRAPH, "graph has no edges");
    std::vector<std::vector<int>> ch(n), pa(n);
    std::vector<std::vector<double>> chw(n);
    for (int e = 0; e < m; ++e) {
        const int a = G->parent[e], b = G->child[e];
        if (a < 0 || a >= n || b < 0 || b >= n)
            return fail(PF_EGRAPH, "edge %d (%d->%d) names a node outside 0..%d", e, a, b, n - 1);
        if (a == b) return fail(PF_EGRAPH, "edge %d is a self loop on %d", e, a);
        if (b == 0) return fail(PF_EGRAPH, "edge %d points into the source", e);
        if (std::find(ch[a].begin(), ch[a].end(), b) != ch[a].end())
            return fail(PF_EGRAPH, "duplicate edge %d->%d", a, b);
        ch[a].push_back(b);
        pa[b].push_back(a);
    }
    for (int e = 0; e < m; ++e) {
        const int a = G->parent[e], b = G->child[e];
        double w = 1.0 / (double)pa[b].size();
        if (G->weight) {
            w = G->weight[e];
            if (!std::isfinite(w) || !(w > 0.0))
                return fail(PF_EGRAPH, "edge %d->%d has weight %g (must be > 0)", a, b, w);
        }
        chw[a].push_back(w);
        (void)b;
    }
    for (int b = 1; b < n; ++b)
        if (pa[b].empty()) return fail(PF_EGRAPH, "node %d has no parent (unreachable)", b);
    if (tree_only) {
        for (int b = 1; b < n; ++b)
            if (pa[b].size() != 1) return fail(PF_EGRAPH, "node %d has %zu parents: not a tree", b, pa[b].size());
        if (G->weight)
            for (int e = 0; e < m; ++e)
                if (G->weight[e] != 1.0) return fail(PF_EGRAPH, "tree edge %d has weight != 1", e);
    }
    // Kahn's algorithm
    std::vector<int> indeg(n), order;
    for (int b = 0; b < n; ++b) indeg[b] = (int)pa[b].size();
    std::vector<int> ready;
    for (int b = 0; b < n; ++b)
        if (!indeg[b]) ready.push_back(b);
    while (!ready.empty()) {
        const int a = ready.back();
        ready.pop_back();
        order.push_back(a);
        for (int c : ch[a])
            if (--indeg[c] == 0) ready.push_back(c);
    }
    if ((int)order.size() != n) return fail(PF_EGRAPH, "label graph has a cycle");
    std::vector<int> leaves;
    for (int a = 1; a < n; ++a)
        if (ch[a].empty()) leaves.push_back(a);
    if ((int)leaves.size() > PF_MAX_LEAVES)
        return fail(PF_EUNSUPPORTED, "%zu end-labels > %d", leaves.size(), PF_MAX_LEAVES);
    // W[a][leaf] by reverse topological order
    std::vector<std::vector<double>> W(n, std::vector<double>(leaves.size(), 0.0));
    for (int i = n - 1; i >= 0; --i) {
        const int a = order[i];
        if (ch[a].empty()) {
            const auto it = std::find(leaves.begin(), leaves.end(), a);
            if (it != leaves.end()) W[a][it - leaves.begin()] = 1.0;
            continue;
        }
        for (size_t j = 0; j < ch[a].size(); ++j)
            for (size_t L = 0; L < leaves.size(); ++L) W[a][L] += chw[a][j] * W[ch[a][j]][L];
    }
    for (size_t L = 0; L < leaves.size(); ++L)
        if (std::fabs(W[0][L] - 1.0) > 1e-9)
            return fail(PF_EGRAPH, "path weights from the source to leaf %d sum to %.12g, not 1",
                        leaves[L], W[0][L]);
    p.nl = (int)leaves.size();
    p.nn = n - 1;
    p.ident = false;
    p.tail = true;
    for (int L = 0; L < p.nl; ++L) p.tail = p.tail && leaves[L] == n - p.nl + L;
    std::memset(&p.w, 0, sizeof p.w);
    p.w.nl = p.nl;
    p.w.nn = p.nn;
    for (int A = 1; A < n; ++A)
        for (int L = 0; L < p.nl; ++L) p.w.w[A - 1][L] = (float)W[A][L];
    return PF_OK;
}

struct Timer {
    std::vector<hipEvent_t> ev;
    ~Timer() {
        for (auto e : ev) hipEventDestroy(e);
    }
};

// Tape geometry: one float32 state (ell, then q) per checkpoint.
struct TapeGeom {
    size_t ell_bytes, slot_bytes;
    int slots;
};

TapeGeom tape_geom(const pf_grid &g, int nl, int nn, int iters, int every) {
    TapeGeom t{};
    const size_t V = (size_t)g.nx * g.ny * g.nz;
    t.ell_bytes = align256((size_t)g.batch * nl * V * 4);
    t.slot_bytes = t.ell_bytes + align256((size_t)g.batch * nn * g.ndim * V * 4);
    t.slots = every > 0 ? (iters + every - 1) / every : 0;
    return t;
}

int check_tape(const Prob &p, const pf_params *P) {
    if (!P->tape) return PF_OK;
    if (P->storage != PF_FP32) return fail(PF_EUNSUPPORTED, "a recorded (differentiable) solve needs fp32 state");
    if (P->ckpt_every < 1) return fail(PF_EINVAL, "ckpt_every must be >= 1");
    if (P->gap_tol != 0.0 || P->warm_start)
        return fail(PF_EINVAL, "a recorded solve runs a fixed iteration budget from the initial state");
    if (!aligned(P->tape, 256)) return fail(PF_EINVAL, "tape is not 256-byte aligned");
    const TapeGeom t = tape_geom(p.g, p.nl, p.nn, P->iters, P->ckpt_every);
    if (P->tape_bytes < (size_t)t.slots * t.slot_bytes)
        return fail(PF_ENOMEM, "tape of %zu bytes < %zu needed", P->tape_bytes, (size_t)t.slots * t.slot_bytes);
    return PF_OK;
}

int run(Prob &p, const pf_params *P, pf_result *R, hipStream_t stream, bool static_ws = false) {
    int tst = check_tape(p, P);
    if (tst != PF_OK) return tst;
    if (P->tape && (P->kernel == PF_KERNEL_FUSED || P->kernel == PF_KERNEL_FUSED2 ||
                    P->kernel == PF_KERNEL_LDS))
        return fail(PF_EUNSUPPORTED, "a recorded solve uses the two-pass kernels");
    const long V = (long)p.g.nx * p.g.ny * p.g.nz;
    // AUTO may take a kernel that ping-pongs the state (tiles, fused passes)
    // unless, on the static scratch, that layout would not fit where the
    // single-state layout of the two-pass kernels does
    const bool auto_pp = P->kernel == PF_KERNEL_AUTO &&
                         !(static_ws && make_layout(p.g, p.nl, p.nn, P->storage, true).total >
                                            (size_t)PF_STATIC_SCRATCH_BYTES);
    // PF_KERNEL_LDS: whole problems per block for batches that fill the GPU
    // (and fit), tiles with ghost zones otherwise
    const bool lds_kind = !P->tape && (P->kernel == PF_KERNEL_LDS ||
                          (P->kernel == PF_KERNEL_AUTO &&
                           (lds_preferred(p.g.ndim, p.nl, p.nn, V, p.g.batch) ||
                            (auto_pp && tile_preferred(p.g.ndim, p.nl, p.nn, V, p.g.batch)))));
    const bool want_lds = lds_kind && lds_preferred(p.g.ndim, p.nl, p.nn, V, p.g.batch);
    const bool want_tile = lds_kind && !want_lds;
    if (want_tile && !tile_supported(p.g.ndim, p.nl, p.nn))
        return fail(PF_EUNSUPPORTED, "LDS-resident iterations serve 2-D problems of up to 8 labels "
                                     "and 16 flows");
    const bool want_fused2 = !P->tape && !lds_kind && (P->kernel == PF_KERNEL_FUSED2 ||
                             (auto_pp && fused2_preferred(p.g.ndim, p.nl, p.nn, p.ident, P->storage)));
    const bool want_fused = want_fused2 || (!P->tape && !lds_kind && (P->kernel == PF_KERNEL_FUSED ||
                            (auto_pp &&
                             any_fused_preferred(p.g.ndim, p.nl, p.nn, p.ident, P->storage, p.tail))));
    if (P->kernel == PF_KERNEL_FUSED && !fused_supported(p.g.ndim, p.nl, p.nn, p.ident))
        return fail(PF_EUNSUPPORTED, "fused kernel unavailable for this problem");
    if (want_fused2 && !fused2_supported(p.g.ndim, p.nl, p.nn, p.ident))
        return fail(PF_EUNSUPPORTED, "two-iteration kernel unavailable for this problem");
    // 3-D label graphs: the fused pass is the flow step of one iteration and
    // the label step of the next (entered with a label pass, left with a flow
    // pass); the label-then-flow fused kernel serves Potts and 2-D graphs
    const bool want_fl = want_fused && !want_fused2 &&
                         flow_label_supported(p.g.ndim, p.nl, p.nn, p.ident);
    const Layout lay = make_layout(p.g, p.nl, p.nn, P->storage, want_fused || want_tile);
    if (static_ws && lay.total > (size_t)PF_STATIC_SCRATCH_BYTES)
        return fail(PF_ENOMEM, "the problem needs %zu bytes of device scratch, more than the %zu "
                               "bytes of the static scratch", lay.total, (size_t)PF_STATIC_SCRATCH_BYTES);
    if (!static_ws && P->workspace_bytes < lay.total)
        return fail(PF_ENOMEM, "workspace of %zu bytes < %zu needed", P->workspace_bytes, lay.total);
    if (!R) return fail(PF_EINVAL, "result is NULL");
    if ((R->u && !aligned(R->u, 4)) || (R->labels && !aligned(R->labels, 4)) ||
        (R->q && !aligned(R->q, 4)) || (R->ell && !aligned(R->ell, 4)))
        return fail(PF_EINVAL, "output pointers must be 4-byte aligned");
    if (R->gap_history && R->gap_history_cap < 0) return fail(PF_EINVAL, "gap_history_cap < 0");

    char *ws = static_cast<char *>(P->workspace);
    if (static_ws) {
        void *sp = nullptr;
        const int st = static_scratch(stream, &sp);
        if (st != PF_OK) return st;
        ws = static_cast<char *>(sp);
    }
    double *results = reinterpret_cast<double *>(ws + lay.results);
    int32_t *flags = reinterpret_cast<int32_t *>(ws + lay.flags);
    double *partials = reinterpret_cast<double *>(ws + lay.partials);
    void *ell[2] = {ws + lay.ell[0], ws + lay.ell[1]};
    void *q[2] = {ws + lay.q[0], ws + lay.q[1]};
    float *consts = reinterpret_cast<float *>(ws + lay.consts);
    const int nd = p.g.ndim;
    const bool ident = p.ident;

    StepArgs a{};
    a.nx = p.g.nx;
    a.ny = p.g.ny;
    a.nz = p.g.nz;
    a.V = p.g.nx * p.g.ny * p.g.nz;
    a.B = p.g.batch;
    a.nl = p.nl;
    a.nn = p.nn;
    a.inv_c = 1.0f / P->c;
    a.ctau = P->c * P->tau;
    a.s_mode = p.s_mode;
    a.D = p.D;
    a.S = p.S;
    a.W = consts + PF_MAX_NODES;
    if (p.s_mode == PF_S_NODE_SCALAR) {
        a.Sp = consts;
        a.s_sb = 0, a.s_sa = 1, a.s_sv = 0;
    } else if (p.s_mode == PF_S_SHARED_FIELD) {
        a.Sp = p.S;
        a.s_sb = a.V, a.s_sa = 0, a.s_sv = 1;
    } else {
        a.Sp = p.S;
        a.s_sb = (int64_t)p.nn * a.V, a.s_sa = a.V, a.s_sv = 1;
    }
    a.ell_in = a.ell_out = ell[0];
    a.q_in = a.q_out = q[0];

    R->iters_done = 0;
    R->gap_history_len = 0;
    R->energy = R->dual = R->gap = NAN;
    R->max_simplex_err = R->max_flow_excess = NAN;
    R->kernel_ms = 0.0;
    R->kernel_timed = 0;

    hipError_t e;
    {
        ConstBlock cb{};
        std::memcpy(cb.s_node, p.s_node, sizeof cb.s_node);
        for (int A = 0; A < PF_MAX_NODES; ++A)
            for (int L = 0; L < PF_MAX_LEAVES; ++L) cb.w[A * PF_MAX_LEAVES + L] = p.w.w[A][L];
        if ((e = launch_upload(cb, consts, stream)) != hipSuccess) return hip_fail(e, "upload");
    }
    if (P->check_inputs) {
        if ((e = launch_check(a, flags, stream)) != hipSuccess) return hip_fail(e, "input check");
        int32_t flag = 0;
        if ((e = hipMemcpyAsync(&flag, flags, sizeof flag, hipMemcpyDeviceToHost, stream)) != hipSuccess)
            return hip_fail(e, "input check copy");
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "input check sync");
        if (flag & 1) return fail(PF_ENONFINITE, "D holds NaN or Inf");
        if (flag & 2) return fail(PF_ENONFINITE, "S holds NaN, Inf or a negative value");
    }
    // iterations per launch sequence (up to the next gap check for the LDS
    // kernels and the flow-then-label passes, two for a pair of the
    // two-iteration kernel) and the state buffer flips they make
    const int kmax_tile = want_tile ? tile_geometry(a.nx, a.ny, a.B, a.nn).k : 1;
    auto step_at = [&](int it) {
        const bool pair = want_fused2 && it + 1 < P->iters &&
                          !(P->gap_every > 0 && (it + 1) % P->gap_every == 0);
        if (want_lds || want_tile || want_fl)
            return P->gap_every > 0 ? std::min(P->iters - it, P->gap_every - it % P->gap_every)
                                    : P->iters - it;
        return pair ? 2 : 1;
    };
    auto flips_of = [&](int step) {
        if (want_tile) return (step + kmax_tile - 1) / kmax_tile;
        if (want_fl) return step - 1;
        return want_fused ? 1 : 0;
    };
    // A fresh solve that runs to its end starts in the buffer that makes it
    // end in the first one (where a warm start looks for the state), so that
    // no copy is needed at the end.
    int cur = 0;
    if (!P->warm_start && !(P->gap_tol > 0.0)) {
        int flips = 0;
        for (int it = 0; it < P->iters;) {
            const int st = step_at(it);
            flips += flips_of(st);
            it += st;
        }
        cur = flips & 1;
    }
    a.ell_in = a.ell_out = ell[cur];
    a.q_in = a.q_out = q[cur];
    if (!P->warm_start) {
        if ((e = launch_init(a, nd, P->storage, -logf((float)p.nl), stream)) != hipSuccess)
            return hip_fail(e, "init");
    }

    auto evaluate = [&](double out[4]) -> int {
        hipError_t err = launch_energy(a, ident, nd, P->storage, partials, results, stream);
        if (err != hipSuccess) return hip_fail(err, "energy");
        if ((err = hipMemcpyAsync(out, results, 4 * sizeof(double), hipMemcpyDeviceToHost,
                                  stream)) != hipSuccess)
            return hip_fail(err, "energy copy");
        if ((err = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(err, "energy sync");
        if (!std::isfinite(out[0]) || !std::isfinite(out[1]))
            return fail(PF_ENONFINITE, "non-finite energy/dual after %d iterations", R->iters_done);
        return PF_OK;
    };

    Timer timer;
    const TapeGeom tg = tape_geom(p.g, p.nl, p.nn, P->iters, P->ckpt_every);
    const size_t n_ell = (size_t)a.B * a.nl * a.V, n_q = (size_t)a.B * a.nn * nd * a.V;
    int timed_iters = 0;
    for (int it = 0; it < P->iters;) {
        // two iterations in one pass unless a gap check falls after the first;
        // the LDS kernels and the flow-then-label passes run every iteration
        // up to the next gap check
        const int step = step_at(it);
        const bool pair = want_fused2 && step == 2;
        if (P->tape && it % P->ckpt_every == 0) {
            char *slot = static_cast<char *>(P->tape) + (size_t)(it / P->ckpt_every) * tg.slot_bytes;
            if ((e = launch_copy_f(static_cast<const float *>(ell[0]), reinterpret_cast<float *>(slot),
                                   n_ell, stream)) != hipSuccess ||
                (e = launch_copy_f(static_cast<const float *>(q[0]),
                                   reinterpret_cast<float *>(slot + tg.ell_bytes), n_q, stream)) != hipSuccess)
                return hip_fail(e, "checkpoint");
        }
        const bool timed = !want_fl && P->timing_stride > 0 &&
                           (want_lds || want_tile || it % P->timing_stride == 0);
        if (timed) {
            hipEvent_t e0, e1;
            if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
                return fail(PF_EHIP, "hipEventCreate failed");
            timer.ev.push_back(e0);
            timer.ev.push_back(e1);
            hipEventRecord(e0, stream);
        }
        if (want_lds) {
            if ((e = launch_lds(a, ident, P->storage, step, stream)) != hipSuccess)
                return hip_fail(e, "LDS-resident iterations");
        } else if (want_tile) {
            // launches of up to k iterations each, ping-pong
            const int kmax = kmax_tile;
            for (int j = 0; j < step; j += kmax) {
                a.ell_in = ell[cur];
                a.q_in = q[cur];
                a.ell_out = ell[1 - cur];
                a.q_out = q[1 - cur];
                if ((e = launch_tile(a, ident, P->storage, std::min(kmax, step - j), stream)) != hipSuccess)
                    return hip_fail(e, "LDS tile iterations");
                cur = 1 - cur;
            }
            a.ell_in = a.ell_out = ell[cur];
            a.q_in = a.q_out = q[cur];
        } else if (want_fl) {
            // label step of iteration it + 1 in place, `step - 1` passes each
            // taking the flows and the labels one iteration further (ping-pong),
            // then the flow step of iteration it + step in place; with timing,
            // the passes starting every timing_stride-th iteration are timed
            a.ell_in = a.ell_out = ell[cur];
            a.q_in = a.q_out = q[cur];
            if ((e = launch_label(a, ident, nd, P->storage, stream)) != hipSuccess)
                return hip_fail(e, "label pass");
            for (int j = 1; j < step; ++j) {
                a.ell_in = ell[cur];
                a.q_in = q[cur];
                a.ell_out = ell[1 - cur];
                a.q_out = q[1 - cur];
                const bool tj = P->timing_stride > 0 && (it + j) % P->timing_stride == 0;
                if (tj) {
                    hipEvent_t e0, e1;
                    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
                        return fail(PF_EHIP, "hipEventCreate failed");
                    timer.ev.push_back(e0);
                    timer.ev.push_back(e1);
                    hipEventRecord(e0, stream);
                }
                if ((e = launch_flow_label(a, P->storage, p.tail, stream)) != hipSuccess)
                    return hip_fail(e, "flow-label pass");
                if (tj) {
                    hipEventRecord(timer.ev.back(), stream);
                    ++timed_iters;
                }
                cur = 1 - cur;
            }
            a.ell_in = a.ell_out = ell[cur];
            a.q_in = a.q_out = q[cur];
            if ((e = launch_flow(a, ident, nd, P->storage, stream)) != hipSuccess)
                return hip_fail(e, "flow pass");
        } else if (want_fused) {
            a.ell_in = ell[cur];
            a.q_in = q[cur];
            a.ell_out = ell[1 - cur];
            a.q_out = q[1 - cur];
            if (pair) {
                if ((e = launch_fused2(a, P->storage, stream)) != hipSuccess)
                    return hip_fail(e, "two-iteration step");
            } else if ((e = launch_fused(a, ident, nd, P->storage, stream)) != hipSuccess) {
                return hip_fail(e, "fused step");
            }
            cur = 1 - cur;
            a.ell_in = a.ell_out;
            a.q_in = a.q_out;
        } else {
            if ((e = launch_label(a, ident, nd, P->storage, stream)) != hipSuccess)
                return hip_fail(e, "label pass");
            if ((e = launch_flow(a, ident, nd, P->storage, stream)) != hipSuccess)
                return hip_fail(e, "flow pass");
        }
        if (timed) {
            hipEventRecord(timer.ev.back(), stream);
            timed_iters += step;
        }
        it += step;
        R->iters_done = it;
        if (P->gap_every > 0 && it % P->gap_every == 0) {
            double r[4];
            const int st = evaluate(r);
            if (st != PF_OK) return st;
            const double gap = r[0] - r[1];
            if (R->gap_history && R->gap_history_len < R->gap_history_cap)
                R->gap_history[R->gap_history_len++] = gap;
            R->energy = r[0];
            R->dual = r[1];
            R->gap = gap;
            R->max_simplex_err = r[2];
            R->max_flow_excess = r[3];
            if (P->gap_tol > 0.0 && gap <= P->gap_tol * std::fabs(r[0])) break;
        }
    }
    if (cur == 1) {
        // bring the state back to the first buffer so that a warm start finds it
        StepArgs c = a;
        c.ell_in = ell[1];
        c.q_in = q[1];
        c.ell_out = ell[0];
        c.q_out = q[0];
        if ((e = launch_copy_state(c, nd, P->storage, stream)) != hipSuccess)
            return hip_fail(e, "state copy");
        a.ell_in = a.ell_out = ell[0];
        a.q_in = a.q_out = q[0];
    }
    if (P->final_energy) {
        double r[4];
        const int st = evaluate(r);
        if (st != PF_OK) return st;
        R->energy = r[0];
        R->dual = r[1];
        R->gap = r[0] - r[1];
        R->max_simplex_err = r[2];
        R->max_flow_excess = r[3];
    }
    if (R->u || R->labels || R->q) {
        if ((e = launch_export(a, nd, P->storage, R->u, R->labels, R->q, stream)) != hipSuccess)
            return hip_fail(e, "export");
    }
    if (R->ell) {
        if ((e = launch_export_ell(a, P->storage, R->ell, stream)) != hipSuccess)
            return hip_fail(e, "export ell");
    }
    if (!timer.ev.empty()) {
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "timing sync");
        double ms = 0.0;
        for (size_t i = 0; i + 1 < timer.ev.size(); i += 2) {
            float t = 0.f;
            if ((e = hipEventElapsedTime(&t, timer.ev[i], timer.ev[i + 1])) != hipSuccess)
                return hip_fail(e, "hipEventElapsedTime");
            ms += t;
        }
        R->kernel_ms = ms;
        R->kernel_timed = timed_iters;
    }
    g_err.clear();
    return PF_OK;
}

// Workspace of a backward call: constants, then ckpt_every float32 segment
// states (the states after the checkpoint; the checkpoint itself is read from
// the tape), two pbar and two lbar buffers (ping-pong for the fused reverse
// kernel) and the per-voxel capacity gradients of node constants.
struct BwdLayout {
    size_t consts, slots, pbar[2], lbar[2], sbar, total;
    TapeGeom tg;
};

BwdLayout bwd_layout(const pf_grid &g, int nl, int nn, int every) {
    BwdLayout L{};
    const size_t V = (size_t)g.nx * g.ny * g.nz;
    L.tg = tape_geom(g, nl, nn, every, every);
    size_t off = 512;
    L.consts = off;
    off = align256(off + sizeof(ConstBlock));
    L.slots = off;
    off += (size_t)every * L.tg.slot_bytes;
    for (int i = 0; i < 2; ++i) {
        L.pbar[i] = off;
        off = align256(off + (size_t)g.batch * nn * g.ndim * V * 4);
    }
    for (int i = 0; i < 2; ++i) {
        L.lbar[i] = off;
        off = align256(off + (size_t)g.batch * nl * V * 4);
    }
    L.sbar = off;
    off = align256(off + (size_t)g.batch * nn * V * 4);
    L.total = off;
    return L;
}

int run_backward(Prob &p, const pf_params *P, const float *grad_ell, float *grad_D, float *grad_S,
                 hipStream_t stream) {
    if (!P->tape) return fail(PF_EINVAL, "backward needs the tape of a recorded solve");
    if (P->storage != PF_FP32) return fail(PF_EUNSUPPORTED, "backward needs fp32 state");
    if (P->ckpt_every < 1) return fail(PF_EINVAL, "ckpt_every must be >= 1");
    const TapeGeom tg = tape_geom(p.g, p.nl, p.nn, P->iters, P->ckpt_every);
    if (!aligned(P->tape, 256) || P->tape_bytes < (size_t)tg.slots * tg.slot_bytes)
        return fail(PF_ENOMEM, "tape smaller than pf_tape_bytes");
    const BwdLayout L = bwd_layout(p.g, p.nl, p.nn, P->ckpt_every);
    if (P->workspace_bytes < L.total)
        return fail(PF_ENOMEM, "backward workspace of %zu bytes < %zu needed", P->workspace_bytes, L.total);
    if (!grad_ell || !grad_D || !grad_S) return fail(PF_EINVAL, "gradient pointers must be set");
    if (!aligned(grad_ell, 4) || !aligned(grad_D, 4) || !aligned(grad_S, 4))
        return fail(PF_EINVAL, "gradient pointers must be 4-byte aligned");
    const int nd = p.g.ndim;
    char *ws = static_cast<char *>(P->workspace);
    float *consts = reinterpret_cast<float *>(ws + L.consts);
    const size_t V = (size_t)p.g.nx * p.g.ny * p.g.nz;
    const size_t n_ell = (size_t)p.g.batch * p.nl * V, n_q = (size_t)p.g.batch * p.nn * nd * V;
    auto slot_ell = [&](int j) { return reinterpret_cast<float *>(ws + L.slots + (size_t)j * L.tg.slot_bytes); };
    auto slot_q = [&](int j) {
        return reinterpret_cast<float *>(ws + L.slots + (size_t)j * L.tg.slot_bytes + L.tg.ell_bytes);
    };
    float *pbar[2] = {reinterpret_cast<float *>(ws + L.pbar[0]), reinterpret_cast<float *>(ws + L.pbar[1])};
    float *lbar[2] = {reinterpret_cast<float *>(ws + L.lbar[0]), reinterpret_cast<float *>(ws + L.lbar[1])};
    // capacity gradient: fields accumulate straight into grad_S ([B][V] shared,
    // [B][nn][V] per node); node constants per voxel first, summed at the end
    const bool s_scalar = p.s_mode == PF_S_NODE_SCALAR;
    float *sbar = s_scalar ? reinterpret_cast<float *>(ws + L.sbar) : grad_S;
    const size_t n_sbar = (size_t)p.g.batch * (p.s_mode == PF_S_SHARED_FIELD ? 1 : p.nn) * V;
    // AUTO: the fused reverse step where it marches 2-D rows, the two-kernel
    // step otherwise (measured faster on MI355X than the tile form, which
    // holds one tile per compute unit at its register count)
    if (P->kernel == PF_KERNEL_FUSED2)
        return fail(PF_EUNSUPPORTED, "no two-iteration reverse kernel");
    if (P->kernel == PF_KERNEL_LDS) return fail(PF_EUNSUPPORTED, "no LDS-resident reverse kernel");
    const bool fused = P->kernel == PF_KERNEL_FUSED ||
                       (P->kernel == PF_KERNEL_AUTO && adj_fused_preferred(nd, p.g.nx, p.nl, p.nn, p.ident));
    if (fused && !adj_fused_supported(nd, p.nl, p.nn, p.ident))
        return fail(PF_EUNSUPPORTED, "fused reverse kernel unavailable for this problem");

    StepArgs a{};
    a.nx = p.g.nx;
    a.ny = p.g.ny;
    a.nz = p.g.nz;
    a.V = (int32_t)V;
    a.B = p.g.batch;
    a.nl = p.nl;
    a.nn = p.nn;
    a.inv_c = 1.0f / P->c;
    a.ctau = P->c * P->tau;
    a.s_mode = p.s_mode;
    a.D = p.D;
    a.S = p.S;
    a.W = consts + PF_MAX_NODES;
    if (p.s_mode == PF_S_NODE_SCALAR) {
        a.Sp = consts;
        a.s_sb = 0, a.s_sa = 1, a.s_sv = 0;
    } else if (p.s_mode == PF_S_SHARED_FIELD) {
        a.Sp = p.S;
        a.s_sb = a.V, a.s_sa = 0, a.s_sv = 1;
    } else {
        a.Sp = p.S;
        a.s_sb = (int64_t)p.nn * a.V, a.s_sa = a.V, a.s_sv = 1;
    }
    hipError_t e;
    {
        ConstBlock cb{};
        std::memcpy(cb.s_node, p.s_node, sizeof cb.s_node);
        for (int A = 0; A < PF_MAX_NODES; ++A)
            for (int Lf = 0; Lf < PF_MAX_LEAVES; ++Lf) cb.w[A * PF_MAX_LEAVES + Lf] = p.w.w[A][Lf];
        if ((e = launch_upload(cb, consts, stream)) != hipSuccess) return hip_fail(e, "upload");
    }
    if ((e = launch_fill(grad_D, n_ell, 0.f, stream)) != hipSuccess ||
        (e = launch_fill(pbar[0], n_q, 0.f, stream)) != hipSuccess ||
        (e = launch_fill(sbar, n_sbar, 0.f, stream)) != hipSuccess ||
        (e = launch_copy_f(grad_ell, lbar[0], n_ell, stream)) != hipSuccess)
        return hip_fail(e, "backward init");
    int cur = 0;
    const bool ident = p.ident;
    const int K = P->iters, k = P->ckpt_every;
    for (int seg = tg.slots - 1; seg >= 0; --seg) {
        const int k0 = seg * k, k1 = std::min(K, k0 + k), m = k1 - k0;
        // state j of the segment: the checkpoint itself (read in place) for
        // j == 0, else the recomputed slot j - 1
        const char *src = static_cast<const char *>(P->tape) + (size_t)seg * tg.slot_bytes;
        auto st_ell = [&](int j) {
            return j == 0 ? const_cast<float *>(reinterpret_cast<const float *>(src)) : slot_ell(j - 1);
        };
        auto st_q = [&](int j) {
            return j == 0 ? const_cast<float *>(reinterpret_cast<const float *>(src + tg.ell_bytes))
                          : slot_q(j - 1);
        };
        // recompute the segment's states out of place; the reverse steps read
        // ell_1 .. ell_m and q_0 .. q_{m-1}, so the last flow step is skipped
        for (int j = 0; j < m; ++j) {
            StepArgs f = a;
            f.ell_in = st_ell(j);
            f.q_in = st_q(j);
            f.ell_out = st_ell(j + 1);
            if ((e = launch_label(f, ident, nd, PF_FP32, stream)) != hipSuccess) return hip_fail(e, "recompute");
            if (j + 1 == m) break;
            f.ell_in = st_ell(j + 1);
            f.q_out = st_q(j + 1);
            if ((e = launch_flow(f, ident, nd, PF_FP32, stream)) != hipSuccess) return hip_fail(e, "recompute");
        }
        for (int step = k1 - 1; step >= k0; --step) {
            const int j = step - k0;
            AdjArgs g{};
            g.q_k = st_q(j);
            g.ell_next = st_ell(j + 1);
            g.sbar = sbar;
            g.sbar_shared = p.s_mode == PF_S_SHARED_FIELD;
            g.dbar = grad_D;
            g.first = step == K - 1;
            g.lbar_in = lbar[cur];
            g.pbar_in = pbar[cur];
            if (fused) {
                g.lbar_out = lbar[1 - cur];
                g.pbar_out = pbar[1 - cur];
                if ((e = launch_adj_fused(a, g, ident, nd, stream)) != hipSuccess)
                    return hip_fail(e, "fused reverse step");
                cur = 1 - cur;
            } else {
                g.lbar_out = lbar[cur];
                g.pbar_out = pbar[cur];
                if ((e = launch_adj_flow(a, g, ident, nd, stream)) != hipSuccess)
                    return hip_fail(e, "adjoint flow");
                if ((e = launch_adj_label(a, g, ident, nd, stream)) != hipSuccess)
                    return hip_fail(e, "adjoint label");
            }
        }
    }
    if (s_scalar && (e = launch_sum_nodes(sbar, p.g.batch, p.nn, V, grad_S, stream)) != hipSuccess)
        return hip_fail(e, "capacity gradient");
    g_err.clear();
    return PF_OK;
}

}  // namespace

extern "C" {

int32_t pf_abi_version(void) { return PF_ABI_VERSION; }

const char *pf_last_error(void) { return g_err.c_str(); }

size_t pf_workspace_bytes(const pf_grid *grid, int32_t n_leaf, int32_t n_node,
                          const pf_params *params) {
    if (check_grid(grid) != PF_OK || !params) return 0;
    if (n_leaf < 1 || n_leaf > PF_MAX_LEAVES || n_node < 1 || n_node > PF_MAX_NODES) return 0;
    if (params->storage < PF_FP32 || params->storage > PF_FP16) return 0;
    // the same sizes serve the identity (Potts) and weighted families
    const long V = (long)grid->nx * grid->ny * grid->nz;
    const bool fused = params->kernel == PF_KERNEL_FUSED || params->kernel == PF_KERNEL_FUSED2 ||
                       (params->kernel == PF_KERNEL_LDS &&
                        !lds_preferred(grid->ndim, n_leaf, n_node, V, grid->batch)) ||
                       (params->kernel == PF_KERNEL_AUTO &&
                        (tile_preferred(grid->ndim, n_leaf, n_node, V, grid->batch) ||
                         any_fused_preferred(grid->ndim, n_leaf, n_node, true, params->storage, true) ||
                         any_fused_preferred(grid->ndim, n_leaf, n_node, false, params->storage, true) ||
                         fused2_preferred(grid->ndim, n_leaf, n_node, true, params->storage)));
    return make_layout(*grid, n_leaf, n_node, params->storage, fused).total;
}

int32_t pf_auto_kernel(const pf_grid *grid, int32_t n_leaf, int32_t n_node, int32_t identity,
                       int32_t storage) {
    if (check_grid(grid) != PF_OK) return -1;
    if (n_leaf < 1 || n_leaf > PF_MAX_LEAVES || n_node < 1 || n_node > PF_MAX_NODES) return -1;
    if (storage < PF_FP32 || storage > PF_FP16) return -1;
    const bool id = identity != 0;
    if (id && n_node != n_leaf) return -1;
    const long V = (long)grid->nx * grid->ny * grid->nz;
    if (lds_preferred(grid->ndim, n_leaf, n_node, V, grid->batch) ||
        tile_preferred(grid->ndim, n_leaf, n_node, V, grid->batch))
        return PF_KERNEL_LDS;
    if (fused2_preferred(grid->ndim, n_leaf, n_node, id, storage)) return PF_KERNEL_FUSED2;
    if (any_fused_preferred(grid->ndim, n_leaf, n_node, id, storage, true)) return PF_KERNEL_FUSED;
    return PF_KERNEL_TWO_PASS;
}

int solve_potts(const pf_grid *grid, int32_t n_labels, const float *D, const float *S,
                int32_t s_mode, const pf_params *params, pf_result *result, void *stream) {
    int st;
    if ((st = check_grid(grid)) != PF_OK) return st;
    if ((st = check_params(params)) != PF_OK) return st;
    if (n_labels < 1) return fail(PF_EINVAL, "n_labels must be >= 1");
    if (n_labels > PF_MAX_LEAVES) return fail(PF_EUNSUPPORTED, "n_labels > %d", PF_MAX_LEAVES);
    Prob p;
    p.g = *grid;
    p.nl = p.nn = n_labels;
    p.ident = true;
    if ((st = check_inputs_common(p, D, S, s_mode)) != PF_OK) return st;
    return run(p, params, result, static_cast<hipStream_t>(stream));
}

static int solve_graph(const pf_grid *grid, const pf_graph *graph, bool tree, const float *D,
                       const float *S, int32_t s_mode, const pf_params *params,
                       pf_result *result, void *stream, bool static_ws = false) {
    int st;
    if ((st = check_grid(grid)) != PF_OK) return st;
    if ((st = check_params(params, static_ws)) != PF_OK) return st;
    Prob p;
    p.g = *grid;
    if ((st = build_graph(graph, tree, p)) != PF_OK) return st;
    if ((st = check_inputs_common(p, D, S, s_mode)) != PF_OK) return st;
    return run(p, params, result, static_cast<hipStream_t>(stream), static_ws);
}

int solve_dagmf_static(const pf_grid *grid, const pf_graph *graph, const float *D, const float *S,
                       int32_t s_mode, const pf_params *params, pf_result *result, void *stream) {
    return solve_graph(grid, graph, false, D, S, s_mode, params, result, stream, true);
}

int solve_dagmf(const pf_grid *grid, const pf_graph *graph, const float *D, const float *S,
                int32_t s_mode, const pf_params *params, pf_result *result, void *stream) {
    return solve_graph(grid, graph, false, D, S, s_mode, params, result, stream);
}

int solve_hmf(const pf_grid *grid, const pf_graph *graph, const float *D, const float *S,
              int32_t s_mode, const pf_params *params, pf_result *result, void *stream) {
    return solve_graph(grid, graph, true, D, S, s_mode, params, result, stream);
}

size_t pf_tape_bytes(const pf_grid *grid, int32_t n_leaf, int32_t n_node, int32_t iters,
                     int32_t ckpt_every) {
    if (check_grid(grid) != PF_OK || iters < 0 || ckpt_every < 1) return 0;
    if (n_leaf < 1 || n_leaf > PF_MAX_LEAVES || n_node < 1 || n_node > PF_MAX_NODES) return 0;
    const TapeGeom t = tape_geom(*grid, n_leaf, n_node, iters, ckpt_every);
    return (size_t)t.slots * t.slot_bytes;
}

size_t pf_backward_workspace_bytes(const pf_grid *grid, int32_t n_leaf, int32_t n_node,
                                   int32_t ckpt_every) {
    if (check_grid(grid) != PF_OK || ckpt_every < 1) return 0;
    if (n_leaf < 1 || n_leaf > PF_MAX_LEAVES || n_node < 1 || n_node > PF_MAX_NODES) return 0;
    return bwd_layout(*grid, n_leaf, n_node, ckpt_every).total;
}

int pf_potts_backward(const pf_grid *grid, int32_t n_labels, const float *D, const float *S,
                         int32_t s_mode, const pf_params *params, const float *grad_ell,
                         float *grad_D, float *grad_S, void *stream) {
    int st;
    if ((st = check_grid(grid)) != PF_OK) return st;
    if ((st = check_params(params)) != PF_OK) return st;
    if (n_labels < 1) return fail(PF_EINVAL, "n_labels must be >= 1");
    if (n_labels > PF_MAX_LEAVES) return fail(PF_EUNSUPPORTED, "n_labels > %d", PF_MAX_LEAVES);
    Prob p;
    p.g = *grid;
    p.nl = p.nn = n_labels;
    p.ident = true;
    if ((st = check_inputs_common(p, D, S, s_mode)) != PF_OK) return st;
    return run_backward(p, params, grad_ell, grad_D, grad_S, static_cast<hipStream_t>(stream));
}

int pf_dagmf_backward(const pf_grid *grid, const pf_graph *graph, const float *D,
                         const float *S, int32_t s_mode, const pf_params *params,
                         const float *grad_ell, float *grad_D, float *grad_S, void *stream) {
    int st;
    if ((st = check_grid(grid)) != PF_OK) return st;
    if ((st = check_params(params)) != PF_OK) return st;
    Prob p;
    p.g = *grid;
    if ((st = build_graph(graph, false, p)) != PF_OK) return st;
    if ((st = check_inputs_common(p, D, S, s_mode)) != PF_OK) return st;
    return run_backward(p, params, grad_ell, grad_D, grad_S, static_cast<hipStream_t>(stream));
}

size_t pf_fullflow_workspace_bytes(const pf_grid *grid, int32_t n_labels) {
    if (check_grid(grid) != PF_OK || !ff_supported(grid->ndim, n_labels)) return 0;
    return ff_layout(*grid, n_labels).total;
}

int solve_potts_fullflow(const pf_grid *grid, int32_t n_labels, const float *D, const float *S,
                         int32_t s_mode, const pf_params *params, pf_result *R, void *stream_) {
    int st;
    if ((st = check_grid(grid)) != PF_OK) return st;
    if ((st = check_params(params)) != PF_OK) return st;
    const pf_params *P = params;
    if (n_labels < 1) return fail(PF_EINVAL, "n_labels must be >= 1");
    if (!ff_supported(grid->ndim, n_labels))
        return fail(PF_EUNSUPPORTED, "the full-flow solver takes at most 16 labels");
    if (P->storage != PF_FP32) return fail(PF_EUNSUPPORTED, "the full-flow solver keeps float32 state");
    if (P->kernel != PF_KERNEL_AUTO && P->kernel != PF_KERNEL_TWO_PASS)
        return fail(PF_EUNSUPPORTED, "the full-flow solver runs its two kernels per iteration only");
    if (P->tape) return fail(PF_EUNSUPPORTED, "the full-flow solver records no tape");
    Prob p;
    p.g = *grid;
    p.nl = p.nn = n_labels;
    p.ident = true;
    if ((st = check_inputs_common(p, D, S, s_mode)) != PF_OK) return st;
    const FFLayout lay = ff_layout(p.g, n_labels);
    if (P->workspace_bytes < lay.total)
        return fail(PF_ENOMEM, "workspace of %zu bytes < %zu needed", P->workspace_bytes, lay.total);
    if (!R) return fail(PF_EINVAL, "result is NULL");
    if (R->ell) return fail(PF_EUNSUPPORTED, "the full-flow state holds no log-labels (ell must be NULL)");
    if ((R->u && !aligned(R->u, 4)) || (R->labels && !aligned(R->labels, 4)) || (R->q && !aligned(R->q, 4)))
        return fail(PF_EINVAL, "output pointers must be 4-byte aligned");
    if (R->gap_history && R->gap_history_cap < 0) return fail(PF_EINVAL, "gap_history_cap < 0");
    hipStream_t stream = static_cast<hipStream_t>(stream_);

    char *ws = static_cast<char *>(P->workspace);
    double *results = reinterpret_cast<double *>(ws + lay.results);
    double *partials = reinterpret_cast<double *>(ws + lay.partials);
    float *consts = reinterpret_cast<float *>(ws + lay.consts);
    const int nd = p.g.ndim;
    StepArgs a{};
    a.nx = p.g.nx;
    a.ny = p.g.ny;
    a.nz = p.g.nz;
    a.V = p.g.nx * p.g.ny * p.g.nz;
    a.B = p.g.batch;
    a.nl = a.nn = n_labels;
    a.inv_c = 1.0f / P->c;
    a.ctau = P->tau;
    a.s_mode = p.s_mode;
    a.D = p.D;
    a.S = p.S;
    a.W = consts + PF_MAX_NODES;
    if (p.s_mode == PF_S_NODE_SCALAR) {
        a.Sp = consts;
        a.s_sb = 0, a.s_sa = 1, a.s_sv = 0;
    } else if (p.s_mode == PF_S_SHARED_FIELD) {
        a.Sp = p.S;
        a.s_sb = a.V, a.s_sa = 0, a.s_sv = 1;
    } else {
        a.Sp = p.S;
        a.s_sb = (int64_t)p.nn * a.V, a.s_sa = a.V, a.s_sv = 1;
    }
    FFArgs f{};
    f.q = reinterpret_cast<float *>(ws + lay.q);
    f.u = reinterpret_cast<float *>(ws + lay.u);
    f.w = reinterpret_cast<float *>(ws + lay.w);
    f.pS = reinterpret_cast<float *>(ws + lay.pS);
    f.c = P->c;
    f.tau = P->tau;

    R->iters_done = 0;
    R->gap_history_len = 0;
    R->energy = R->dual = R->gap = NAN;
    R->max_simplex_err = R->max_flow_excess = NAN;
    R->kernel_ms = 0.0;
    R->kernel_timed = 0;
    hipError_t e;
    {
        ConstBlock cb{};
        std::memcpy(cb.s_node, p.s_node, sizeof cb.s_node);
        if ((e = launch_upload(cb, consts, stream)) != hipSuccess) return hip_fail(e, "upload");
    }
    if (P->check_inputs) {
        int32_t *flags = reinterpret_cast<int32_t *>(ws + lay.results + 64);
        if ((e = launch_check(a, flags, stream)) != hipSuccess) return hip_fail(e, "input check");
        int32_t flag = 0;
        if ((e = hipMemcpyAsync(&flag, flags, sizeof flag, hipMemcpyDeviceToHost, stream)) != hipSuccess)
            return hip_fail(e, "input check copy");
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "input check sync");
        if (flag & 1) return fail(PF_ENONFINITE, "D holds NaN or Inf");
        if (flag & 2) return fail(PF_ENONFINITE, "S holds NaN, Inf or a negative value");
    }
    if (!P->warm_start && (e = launch_ff_init(a, f, nd, stream)) != hipSuccess)
        return hip_fail(e, "full-flow init");
    auto evaluate = [&](double out[4]) -> int {
        hipError_t err = launch_ff_energy(a, f, nd, partials, results, stream);
        if (err != hipSuccess) return hip_fail(err, "full-flow energy");
        if ((err = hipMemcpyAsync(out, results, 4 * sizeof(double), hipMemcpyDeviceToHost,
                                  stream)) != hipSuccess)
            return hip_fail(err, "energy copy");
        if ((err = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(err, "energy sync");
        if (!std::isfinite(out[0]) || !std::isfinite(out[1]))
            return fail(PF_ENONFINITE, "non-finite energy/dual after %d iterations", R->iters_done);
        return PF_OK;
    };
    Timer timer;
    int timed = 0;
    for (int it = 0; it < P->iters; ++it) {
        const bool tj = P->timing_stride > 0 && it % P->timing_stride == 0;
        if (tj) {
            hipEvent_t e0, e1;
            if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
                return fail(PF_EHIP, "hipEventCreate failed");
            timer.ev.push_back(e0);
            timer.ev.push_back(e1);
            hipEventRecord(e0, stream);
        }
        if ((e = launch_ff_iteration(a, f, nd, stream)) != hipSuccess)
            return hip_fail(e, "full-flow iteration");
        if (tj) {
            hipEventRecord(timer.ev.back(), stream);
            ++timed;
        }
        R->iters_done = it + 1;
        if (P->gap_every > 0 && (it + 1) % P->gap_every == 0) {
            double r[4];
            if ((st = evaluate(r)) != PF_OK) return st;
            const double gap = r[0] - r[1];
            if (R->gap_history && R->gap_history_len < R->gap_history_cap)
                R->gap_history[R->gap_history_len++] = gap;
            R->energy = r[0], R->dual = r[1], R->gap = gap;
            R->max_simplex_err = r[2], R->max_flow_excess = r[3];
            if (P->gap_tol > 0.0 && gap <= P->gap_tol * std::fabs(r[0])) break;
        }
    }
    if (P->final_energy) {
        double r[4];
        if ((st = evaluate(r)) != PF_OK) return st;
        R->energy = r[0], R->dual = r[1], R->gap = r[0] - r[1];
        R->max_simplex_err = r[2], R->max_flow_excess = r[3];
    }
    if ((R->u || R->labels || R->q) &&
        (e = launch_ff_export(a, f, nd, R->u, R->labels, R->q, stream)) != hipSuccess)
        return hip_fail(e, "full-flow export");
    if (!timer.ev.empty()) {
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "timing sync");
        double ms = 0.0;
        for (size_t i = 0; i + 1 < timer.ev.size(); i += 2) {
            float t = 0.f;
            if ((e = hipEventElapsedTime(&t, timer.ev[i], timer.ev[i + 1])) != hipSuccess)
                return hip_fail(e, "hipEventElapsedTime");
            ms += t;
        }
        R->kernel_ms = ms;
        R->kernel_timed = timed;
    }
    g_err.clear();
    return PF_OK;
}

int solve_ishikawa(const pf_grid *grid, int32_t n_labels, const float *D, const float *S,
                   int32_t s_mode, const pf_params *params, pf_result *result, void *stream) {
    int st;
    if ((st = check_grid(grid)) != PF_OK) return st;
    if ((st = check_params(params)) != PF_OK) return st;
    if (n_labels < 2) return fail(PF_EINVAL, "the Ishikawa chain needs n_labels >= 2");
    if (n_labels > PF_MAX_LEAVES) return fail(PF_EUNSUPPORTED, "n_labels > %d", PF_MAX_LEAVES);
    if (params->kernel == PF_KERNEL_FUSED2 || (params->kernel == PF_KERNEL_FUSED && grid->ndim != 3))
        return fail(PF_EUNSUPPORTED, "no %s kernel for the Ishikawa chain%s",
                    params->kernel == PF_KERNEL_FUSED2 ? "two-iteration" : "fused",
                    params->kernel == PF_KERNEL_FUSED2 ? "" : " in 2-D");
    Prob p;
    p.g = *grid;
    p.nl = n_labels;
    p.nn = n_labels - 1;
    p.ident = false;
    std::memset(&p.w, 0, sizeof p.w);
    p.w.nl = p.nl;
    p.w.nn = p.nn;
    // flow j (of label L_{j+1}) drives every label L_i with i >= j + 1
    for (int j = 0; j < p.nn; ++j)
        for (int L = j + 1; L < p.nl; ++L) p.w.w[j][L] = 1.0f;
    if ((st = check_inputs_common(p, D, S, s_mode)) != PF_OK) return st;
    pf_params P2 = *params;
    const long V = (long)p.g.nx * p.g.ny * p.g.nz;
    if (P2.kernel == PF_KERNEL_AUTO) {
        if (lds_preferred(p.g.ndim, p.nl, p.nn, V, p.g.batch) ||
            tile_preferred(p.g.ndim, p.nl, p.nn, V, p.g.batch))
            P2.kernel = PF_KERNEL_LDS;
        else if (any_fused_preferred(p.g.ndim, p.nl, p.nn, false, P2.storage, p.tail))
            P2.kernel = PF_KERNEL_FUSED;
        else
            P2.kernel = PF_KERNEL_TWO_PASS;
    }
    return run(p, &P2, result, static_cast<hipStream_t>(stream));
}

}  // extern "C"
