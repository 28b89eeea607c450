// Launchers of the adjoint kernels (qlg_adjoint_kernels.hip).
#pragma once

#include "qlg_internal.hpp"

namespace qlg {

hipError_t launch_sub_potential(int dtype, const void* in, void* out, const LaunchGeom& g, double tg0, double tg1,
                                double tg25, hipStream_t st);
hipError_t launch_sub_iprime(int dtype, const void* in, void* out, const LaunchGeom& g, int axis, int qb,
                             hipStream_t st);
hipError_t launch_sub_iprime_adj(const void* in, void* out, const LaunchGeom& g, int axis, int qb, hipStream_t st);
// lam <- (dU)^H lam at z; acc[0..2] += dL/dg (part: nchunks x 3 doubles of scratch)
hipError_t launch_sub_vjp(int dtype, const void* z, void* lam, const LaunchGeom& g, double theta, double g0,
                          double g1, double g2, double* part, double* acc, hipStream_t st);
// energy objective: canonical complex128 cotangent + chunk partials [nchunks][4]
hipError_t launch_energy_grad(int dtype, int ndim, const void* state, void* lam, const LaunchGeom& g, double eps,
                              double g0, double g1, double g2, double* part, hipStream_t st);
// fidelity objective: partials [nchunks][3], per-instance overlaps ov[nbatch][3]
hipError_t launch_fidelity_grad(int dtype, const void* state, const void* target, void* lam, const LaunchGeom& g,
                                double meas, double* part, double* ov, hipStream_t st);
hipError_t launch_lam_layout(bool to_planes, const void* src, void* dst, const LaunchGeom& g, hipStream_t st);
hipError_t launch_zero(double* p, int n, hipStream_t st);

}  // namespace qlg
