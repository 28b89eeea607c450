// Internal declarations shared by the kernels (qlg_kernels.hip) and the C ABI
// implementation (qlg_api.cpp).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qlg.h"

namespace qlg {

// One lattice instance inside a batch.  Offsets are in complex elements.
struct InstDesc {
  int64_t off;        // first element of the instance's 10 qubit planes in one state copy
  int64_t psi_off;    // first element of the instance in the canonical psi layout
  int64_t qb_off;     // first element of the instance in the canonical qubits layout
  int64_t stride;     // plane stride (>= sites, multiple of 64)
  int32_t nx, ny, nz; // extents (ny = 1 in 1D, nz = 1 in 1D and 2D)
  int32_t sites;      // nx * ny * nz
  int32_t tile_begin; // first global wave tile of the fused step (3D: of its y-x pass)
  int32_t ntx, nty;   // tiles along x and bands along y (nty = 1 in 1D); 3D: ntx * nty * nz tiles
  int32_t tile_begin_z;  // 3D z pass: first tile, 64-column tiles along x, bands along z,
  int32_t ntx_z, ntz;    // ntx_z * ntz * ny tiles
  int32_t chunk_begin;// first 256-site chunk for elementwise / reduction kernels
  int32_t nchunks;
};

constexpr int kChunk = 256;      // sites per chunk of the elementwise / reduction kernels
constexpr int kNObs = 10;        // norm_q, norm_psi, pop[5], e_kin, e_pot, spare
constexpr int kRecord = 16;      // doubles per instance in an observables record
constexpr int kLanes = 64;       // wavefront width on gfx950
constexpr int kHalo2D = 4;       // x halo of the 2D kernel (4 I' per axis per step)
constexpr int kValid2D = kLanes - 2 * kHalo2D;

struct LaunchGeom {
  const InstDesc* inst;        // device [nbatch]
  const int32_t* tile2inst;    // device [ntiles]
  const int32_t* chunk2inst;   // device [nchunks]
  const int32_t* tile2inst_z;  // device [ntiles_z], 3D z pass
  int32_t ntiles, nchunks, nbatch, ntiles_z;
};

// The psi-independent diagonal term (V(x) + mu) psi_m of the equation of motion
// (Sec. II, "Additional terms"): V per site in the canonical scalar layout (FP64,
// [instance][y][x]; nullptr: none) and a uniform mu.  theta is the interleaved
// angle eps^2 / (4 d); the plain split uses eps^2.
struct ExtPot {
  const double* V = nullptr;
  double mu = 0.0;
  double theta = 0.0;
  bool on() const { return V != nullptr || mu != 0.0; }
};

// Kernel launchers (qlg_kernels.hip).  All return the hipError_t of the launch.
// dtype: 0 = complex64, 1 = complex128.  Angles are theta*g0, theta*g1, theta*g2/5.
// ev0/ev1 (optional): events the dispatch packet itself stamps at kernel start/end.
// split: where the two qubit amplitudes of a site live: 0 = one lane holds both
// (k_step1d, 64-site tiles, steps <= 7); 1 = two wavefronts (k_step1d_pair, 64-site
// tiles, steps <= 7); 2 = two neighbouring lanes (k_step1d_lanes, 32-site tiles, steps <= 3).
constexpr int kLaneTileSites = 32;
hipError_t launch_step1d(int dtype, int steps, int split, bool plain, bool overlap, const void* in, void* out,
                         const LaunchGeom& g, double tg0, double tg1, double tg25, const ExtPot& ext,
                         double* ovpart, hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Part of a step that one launch of the 2D kernel runs: all four y (or z) stages, then
// the x half unless it is a z pass (kWhole); or the y half over two launches, kYFirst (the
// two stages that move qubit b) and kYSecond (the two that move qubit a, then the x half),
// each with a two-stage row pipeline: half the LDS per wavefront.
enum StepPart : int { kWhole = 0, kYFirst = 1, kYSecond = 2 };
// 2D step, or one pass of a 3D step: zpass = the four z substeps only (rows along z,
// 64-column tiles, the 3D z-pass tile table); otherwise the y and x substeps of each
// z plane.  full_factor: theta of the plain split's single U over the interleaved theta
// (4 ndim); plain_u: this pass applies that U (2D, 3D z pass).  prev (may equal out):
// the state before the step, for the overlap partials.
hipError_t launch_step2d(int dtype, bool plain, bool overlap, int tile_rows, bool zpass, bool plain_u, int part,
                         double full_factor, const void* in, void* out, const void* prev, const LaunchGeom& g,
                         double tg0, double tg1, double tg25, const ExtPot& ext, double* ovpart,
                         hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_set_psi(int dtype, const void* psi, void* state, const LaunchGeom& g, hipStream_t st);
hipError_t launch_get_psi(int dtype, const void* state, void* psi, const LaunchGeom& g, hipStream_t st);
hipError_t launch_set_qubits(int dtype, const void* qb, void* state, const LaunchGeom& g, hipStream_t st);
hipError_t launch_get_qubits(int dtype, const void* state, void* qb, const LaunchGeom& g, hipStream_t st);
// Per-chunk partial sums of the kNObs observables into part[nchunks][kNObs]; the
// potential energy density includes (V + mu) n.
hipError_t launch_observables(int dtype, int ndim, const void* state, const LaunchGeom& g, double g0,
                              double g1, double g2, const ExtPot& ext, double* part, hipStream_t st);
// Per-instance record rec[nbatch][kRecord] from the chunk partials, the per-tile
// overlap partials (ovpart may be null) and a reference record (ref may be null).
hipError_t launch_record(const LaunchGeom& g, const double* part, const double* ovpart, const double* ref,
                         double* rec, int64_t step, hipStream_t st);

// Host checks of a parameter block shared by every entry point that takes one (no
// device call, no allocation); *msg receives a static description of the failure.
qlg_status validate_params(const qlg_params* p, const char** msg);
// Observables records (kRecord doubles per instance, written by k_reduce_record) to
// qlg_obs values; false if a record is non-finite or drifted (no allocation).
bool decode_record_values(const qlg_params& p, const double* rec, int64_t nrec, qlg_obs* out);

}  // namespace qlg
