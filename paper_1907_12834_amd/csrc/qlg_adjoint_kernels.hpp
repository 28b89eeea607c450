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
// substep input z; dg partials per wavefront (a quarter of a chunk) into part[4 nchunks][3]
// (no accumulation).
hipError_t launch_sub_adj(int dtype, const void* z, const void* lam_in, void* lam_out, const LaunchGeom& g, int axis,
                          int qb, double theta, double g0, double g1, double g2, const ExtPot& ext, double* part,
                          hipStream_t st);
// The four adjoint substeps along x of one step in one launch (k_adj_x4): z[0..3] are the
// recorded inputs of substeps k0 + 3, k0 + 2, k0 + 1, k0 (the order they are undone in);
// nwaves = xpre[nbatch] wavefronts of 56 columns of one row; one dg partial per wavefront
// into part[nwaves][3] (no accumulation).
hipError_t launch_adj_x4(int dtype, const void* const z[4], const void* lam_in, void* lam_out, const LaunchGeom& g,
                         const int* xpre, int nwaves, double theta, double g0, double g1, double g2,
                         const ExtPot& ext, double* part, hipStream_t st);
// The chain links that apply x kinetic factors, fused (k_chain_x4): links (j, nsub - 3 ..
// nsub - 1) and, when rec[3] is not null, (j + 1, 0); rec[i] receives the input of the
// link's U, out the state after the last.  Tiles as launch_adj_x4's.
hipError_t launch_chain_x4(int dtype, const void* in, void* out, void* const rec[4], const LaunchGeom& g,
                           const int* xpre, int nwaves, double tg0, double tg1, double tg25, const ExtPot& ext,
                           double theta, hipStream_t st);
// xpre[0..nbatch]: prefix sums over the instances of ceil(nx / 56) ny nz (device table)
hipError_t launch_x4_prefix(const LaunchGeom& g, int* xpre, hipStream_t st);
// acc[0..2] += sum of nparts consecutive 3-vectors of part (fixed order)
hipError_t launch_dg_accumulate(const double* part, int nparts, double* acc, hipStream_t st);
// The same for many partials: kDgBlocks workgroups sum contiguous ranges of part into
// red[kDgBlocks][3] (fixed order), then one workgroup adds those to acc in order.
constexpr int kDgBlocks = 256;
hipError_t launch_dg_reduce(const double* part, int64_t nparts, double* red, double* acc, hipStream_t st);
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
