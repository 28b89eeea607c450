// Launchers of the per-site diagnostic kernels (qlg_diag_kernels.hip).
// Internal to the library; the public entry points are qlg_fields and
// qlg_vorticity in include/qlg.h.
#pragma once

#include "qlg_internal.hpp"

namespace qlg {

// n, F_par, F_perp, |A00| of every site (FP64, canonical scalar layout
// [instance][y][x]); a NULL output is skipped.  dtype: 0 = complex64, 1 = complex128.
hipError_t launch_fields(int dtype, const void* state, const LaunchGeom& g, double* n, double* f_par,
                         double* f_perp, double* a00, hipStream_t st);

// Vorticity (FP64) and plaquette winding numbers (int32) of component m of one
// instance, written at the instance's place in the canonical scalar layout; a
// NULL output is skipped.  2D: one component.  3D: the three plane families,
// normal to x, y and z, component c at offset c * component_stride, from one
// fused pass over the lattice.
hipError_t launch_vorticity(int dtype, int ndim, const void* state, const InstDesc& d, int m, double* omega,
                            int32_t* winding, int64_t component_stride, hipStream_t st);

// The non-zero entries of a winding field (canonical scalar layout) as an ordered
// list, k < capacity: 2D out[k] = {instance, y, x, winding}; 3D, whose winding
// field holds the three plane families at component_stride from each other,
// out[k] = {instance, family, z, y, x, winding} in (family, instance, z, y, x)
// order.  *total (device) receives the number of cores.  counts: nchunks int64
// of workspace per family.
hipError_t launch_vortex_cores(const int32_t* winding, const LaunchGeom& g, int ndim, int64_t component_stride,
                               int64_t* counts, int32_t* out, int64_t capacity, int64_t* total, hipStream_t st);

}  // namespace qlg
