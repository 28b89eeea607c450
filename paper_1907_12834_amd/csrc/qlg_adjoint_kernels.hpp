// Launchers of the adjoint kernels (qlg_adjoint_kernels.hip).
#pragma once

#include "qlg_internal.hpp"

namespace qlg {

// One link of the recorded forward chain: z = I'_{axis,qb}(in) (z = in when axis < 0),
// rec <- z when rec is not null, out <- U(z) with angles (tg0, tg1, tg25) when with_u, else z.
// ext (V, mu) with theta: the potential's per-site phase theta (V + mu) inside U.
hipError_t launch_chain(int dtype, const void* in, void* out, void* rec, const LaunchGeom& g, int axis, int qb,
                        bool with_u, double tg0, double tg1, double tg25, const ExtPot& ext, double theta,
                        hipStream_t st);
hipError_t launch_sub_iprime_adj(const void* in, void* out, const LaunchGeom& g, int axis, int qb, hipStream_t st);
// lam <- (dU)^H lam at z; acc[0..2] += dL/dg (part: nchunks x 3 doubles of scratch)
hipError_t launch_sub_vjp(int dtype, const void* z, void* lam, const LaunchGeom& g, double theta, double g0,
                          double g1, double g2, const ExtPot& ext, double* part, double* acc, hipStream_t st);
// Fused adjoint substep of the interleaved split: lam_out = (dU)^H I'_{axis,qb}^H lam_in at the
// substep input z; per-chunk dg partials into part[nchunks][3] (no accumulation).
hipError_t launch_sub_adj(int dtype, const void* z, const void* lam_in, void* lam_out, const LaunchGeom& g, int axis,
                          int qb, double theta, double g0, double g1, double g2, const ExtPot& ext, double* part,
                          hipStream_t st);
// acc[0..2] += sum of nparts consecutive 3-vectors of part (fixed order)
hipError_t launch_dg_accumulate(const double* part, int nparts, double* acc, hipStream_t st);
// energy objective: canonical complex128 cotangent + chunk partials [nchunks][4]
hipError_t launch_energy_grad(int dtype, int ndim, const void* state, void* lam, const LaunchGeom& g, double eps,
                              double g0, double g1, double g2, const ExtPot& ext, double* part, hipStream_t st);
// fidelity objective: partials [nchunks][3], per-instance overlaps ov[nbatch][3]
hipError_t launch_fidelity_grad(int dtype, const void* state, const void* target, void* lam, const LaunchGeom& g,
                                double meas, double* part, double* ov, hipStream_t st);
hipError_t launch_lam_layout(bool to_planes, const void* src, void* dst, const LaunchGeom& g, hipStream_t st);
// dpsi = (lambda_a + lambda_b) / 2: adjoint of the encoding, complex128 canonical layouts
hipError_t launch_encode_adj(const void* lam, void* dpsi, const LaunchGeom& g, hipStream_t st);
hipError_t launch_zero(double* p, int n, hipStream_t st);

}  // namespace qlg
