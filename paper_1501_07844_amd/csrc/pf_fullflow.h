// Internal interface of the full-flow Potts kernels (pf_fullflow.hip), the
// counterpart the pseudo-flow method is measured against.  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "pf_internal.h"

namespace pf {

// Full-flow state, float32, caller's workspace: spatial flows q
// [B][n][nd][V], labels (the multipliers of flow conservation) u [B][n][V],
// the flow-step driver w_L = div q_L - p_S + p_L - u_L / c [B][n][V] (it
// replaces the sink flows, which every iteration recomputes), and the source
// flow pS [B][V].  The sizes, data terms and capacities come from StepArgs
// (nl = nn = n labels, inv_c = 1/c, ctau = the flow step tau).
struct FFArgs {
    float *q;
    float *u;
    float *w;
    float *pS;
    float c;        // penalty of the augmented Lagrangian
    float tau;      // spatial-flow step
};

struct FFLayout {
    size_t results, partials, consts, q, u, w, pS, total;
};
FFLayout ff_layout(const pf_grid &g, int n);

bool ff_supported(int nd, int n);
hipError_t launch_ff_init(const StepArgs &a, const FFArgs &f, int nd, hipStream_t s);
// one iteration: the spatial-flow step, then the sink, source and label steps
hipError_t launch_ff_iteration(const StepArgs &a, const FFArgs &f, int nd, hipStream_t s);
// float64 energy of the clipped, renormalised labels, the pseudo-flow dual of
// q, max |sum_L u_L - 1| and max |q| - S: results[0..3]
hipError_t launch_ff_energy(const StepArgs &a, const FFArgs &f, int nd, double *partials,
                            double *results, hipStream_t s);
hipError_t launch_ff_export(const StepArgs &a, const FFArgs &f, int nd, float *u, int32_t *labels,
                            float *q, hipStream_t s);

}  // namespace pf
