// Per-site diagnostics of a QLG state: the spin-density fields of Sec. III
// eq. (cmap) and the lattice vorticity of one hyperfine component (Sec. VI,
// "Calculating quantum vorticity on a lattice").
//
// Both read psi = a + b formed in the state's own precision (the value
// qlg_get_psi returns) and work in FP64 from there.
#include "qlg_diag.hpp"
#include "qlg_math.hpp"

namespace qlg {
namespace {

constexpr double kPi = 3.141592653589793;
constexpr double kTwoPi = 2.0 * kPi;

// ---------------------------------------------------------------------------
// Fields: n, F_par = F_z, F_perp = |F_+|, |A00| = |sigma| / sqrt(5)
// ---------------------------------------------------------------------------
// One thread per site, 256-site chunks of one instance per workgroup (the
// chunk table of the elementwise kernels).  With F_+ = sum_m
// sqrt(6 - m(m+1)) psi*_{m+1} psi_m, F_x = Re F_+ and F_y = Im F_+, so
// F_perp = sqrt(F_x^2 + F_y^2) = |F_+|; sigma = 2 psi_2 psi_-2 - 2 psi_1 psi_-1
// + psi_0^2 is the singlet pair amplitude psi^T S psi.
// One amplitude read once and not again by this kernel: loaded with the
// non-temporal hint, which keeps the ten qubit planes streaming through the
// caches without displacing lines still to be read.
template <typename T>
__device__ __forceinline__ cx<T> load_stream(const cx<T>* p) {
  return cx<T>{__builtin_nontemporal_load(&p->re), __builtin_nontemporal_load(&p->im)};
}

template <typename T>
__global__ __launch_bounds__(kChunk) void k_fields(const cx<T>* __restrict__ st, LaunchGeom g,
                                                  double* __restrict__ n_out, double* __restrict__ fpar_out,
                                                  double* __restrict__ fperp_out, double* __restrict__ a00_out) {
  const InstDesc d = g.inst[g.chunk2inst[blockIdx.x]];
  const int s = (blockIdx.x - d.chunk_begin) * kChunk + threadIdx.x;
  if (s >= d.sites) return;
  cx<double> p[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const cx<T> v = load_stream(st + d.off + m * d.stride + s) + load_stream(st + d.off + (5 + m) * d.stride + s);
    p[m] = cx<double>{(double)v.re, (double)v.im};
  }
  double q[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) q[m] = p[m].re * p[m].re + p[m].im * p[m].im;
  const int64_t o = d.psi_off / 5 + s;  // the canonical scalar layout [instance][y][x]
  if (n_out) n_out[o] = q[0] + q[1] + q[2] + q[3] + q[4];
  if (fpar_out) fpar_out[o] = 2.0 * (q[0] - q[4]) + (q[1] - q[3]);
  if (fperp_out) {
    const double r6 = 2.449489742783178;  // sqrt(6)
    cx<double> fp = 2.0 * cmulc(p[0], p[1]);
    fp = rfma(r6, cmulc(p[1], p[2]), fp);
    fp = rfma(r6, cmulc(p[2], p[3]), fp);
    fp = rfma(2.0, cmulc(p[3], p[4]), fp);
    fperp_out[o] = sqrt(fp.re * fp.re + fp.im * fp.im);
  }
  if (a00_out) {
    cx<double> sg = p[2] * p[2];
    sg = rfma(2.0, p[0] * p[4], sg);
    sg = rfma(-2.0, p[1] * p[3], sg);
    a00_out[o] = sqrt(sg.re * sg.re + sg.im * sg.im) * 0.4472135954999579;  // 1/sqrt(5)
  }
}

// ---------------------------------------------------------------------------
// Vorticity and plaquette windings of component m (2D, periodic)
// ---------------------------------------------------------------------------
// Phase S = arg psi_m (0 where psi_m is exactly zero).  Velocities are the
// central differences v_x = wrap(S(x+1) - S(x-1)) / 2, v_y likewise, each
// difference reduced to (-pi, pi]; omega is their central-difference curl
//   omega = (v_y(x+1, y) - v_y(x-1, y) - v_x(x, y+1) + v_x(x, y-1)) / 2,
// which needs S only at the four diagonal neighbours.  The winding number of
// the plaquette with corner (x, y) is the sum of the wrapped differences
// around (x, y) -> (x+1, y) -> (x+1, y+1) -> (x, y+1), over 2 pi.
//
// A workgroup of 256 threads owns a 64 x 16 tile of outputs.  It loads psi_m
// of the tile and a one-site periodic halo, 66 x 18 sites (1.16 per output),
// issuing every load of a thread before the first atan2, then stores the
// phases in LDS; every thread then reads its neighbours from there.
// Floating-point contraction is off so that each difference, product and sum
// rounds once, in the order written.  The kernel takes its plane as a family
// (u and v axes with their extents and site strides, planes along a third
// axis); a 2D lattice is the one family u = x, v = y.
struct PlaneFamily {
  int32_t nu, nv, np;
  int64_t su, sv, sp;
};

constexpr int kVortW = 64, kVortH = 16, kVortThreads = 256;
constexpr int kVortLW = kVortW + 2, kVortLH = kVortH + 2;
constexpr int kVortLoads = (kVortLW * kVortLH + kVortThreads - 1) / kVortThreads;

__device__ __forceinline__ double phase_of(double re, double im) {
  return (re == 0.0 && im == 0.0) ? 0.0 : atan2(im, re);
}

// d is a difference of two phases in [-pi, pi]: one add or subtract of 2 pi
// brings it to (-pi, pi]
__device__ __forceinline__ double wrap_pi(double dlt) {
  return dlt > kPi ? dlt - kTwoPi : (dlt <= -kPi ? dlt + kTwoPi : dlt);
}

// coordinate c in [-1, n + 65) brought to [0, n); tiles wider than the
// lattice (n < 66) wrap more than once
__device__ __forceinline__ uint32_t wrap_coord(int64_t c, int32_t n) {
  if (c < 0) c += n;
  uint32_t u = (uint32_t)c;
  if (u >= (uint32_t)n) u = u - (uint32_t)n < (uint32_t)n ? u - (uint32_t)n : u % (uint32_t)n;
  return u;
}

// The curl at (u, v) of a plane from the phases at its four diagonal neighbours
// pp = S(u+1, v+1), pm = S(u+1, v-1), mp = S(u-1, v+1), mm = S(u-1, v-1): the
// velocities v_v(u+1), v_v(u-1), v_u(v+1), v_u(v-1) as wrapped half differences,
// then (v_v(u+1) - v_v(u-1) - v_u(v+1) + v_u(v-1)) / 2 in that order.
__device__ __forceinline__ double curl_of(double pp, double pm, double mp, double mm) {
#pragma clang fp contract(off)
  const double vv_p = wrap_pi(pp - pm) / 2.0;
  const double vv_m = wrap_pi(mp - mm) / 2.0;
  const double vu_p = wrap_pi(pp - mp) / 2.0;
  const double vu_m = wrap_pi(pm - mm) / 2.0;
  return (((vv_p - vv_m) - vu_p) + vu_m) / 2.0;
}

// The winding of the plaquette (u, v) -> (u+1, v) -> (u+1, v+1) -> (u, v+1)
// from the phases at its corners in that order.  The four unwrapped differences
// sum to zero and each reduction adds a multiple of the double 2 pi, so circ is a
// multiple of 2 pi to within a few units in the last place: circ / (2 pi) and
// circ * (1 / (2 pi)) both lie within 1e-14 of the same integer and round to it.
__device__ __forceinline__ int32_t winding_of(double s00, double s10, double s11, double s01) {
#pragma clang fp contract(off)
  constexpr double kInvTwoPi = 0.15915494309189535;
  const double circ = ((wrap_pi(s10 - s00) + wrap_pi(s11 - s10)) + wrap_pi(s01 - s11)) + wrap_pi(s00 - s01);
  return (int32_t)rint(circ * kInvTwoPi);
}

template <typename T>
__global__ __launch_bounds__(kVortThreads) void k_vorticity(const cx<T>* __restrict__ st, InstDesc d,
                                                           PlaneFamily f, int m, int64_t block0,
                                                           double* __restrict__ omega_out,
                                                           int32_t* __restrict__ wind_out) {
#pragma clang fp contract(off)
  __shared__ double S[kVortLH][kVortLW];
  // tile (u0, v0) of plane p: the x, y of the comments above are u, v of the family
  const int64_t ntu = (f.nu + kVortW - 1) / kVortW, ntv = (f.nv + kVortH - 1) / kVortH;
  // the workgroups one XCD runs (every eighth in launch order) take consecutive
  // tiles, so the halo lines shared by neighbouring tiles meet in one L2
  int64_t blk = blockIdx.x;
  if (gridDim.x % 8 == 0) blk = (blk % 8) * (gridDim.x / 8) + blk / 8;
  blk += block0;
  const int64_t tq = blk / ntu;
  const int64_t x0 = (blk % ntu) * kVortW, y0 = (tq % ntv) * kVortH, pofs = (tq / ntv) * f.sp;
  const cx<T>* pa = st + d.off + (int64_t)m * d.stride + pofs;
  const cx<T>* pb = st + d.off + (int64_t)(5 + m) * d.stride + pofs;
  cx<T> v[kVortLoads];
#pragma unroll
  for (int r = 0; r < kVortLoads; ++r) {
    const int i = threadIdx.x + r * kVortThreads;
    if (i < kVortLH * kVortLW) {
      const int ly = i / kVortLW, lx = i - ly * kVortLW;
      const int64_t s = (int64_t)wrap_coord(y0 - 1 + ly, f.nv) * f.sv + (int64_t)wrap_coord(x0 - 1 + lx, f.nu) * f.su;
      v[r] = pa[s] + pb[s];
    }
  }
#pragma unroll
  for (int r = 0; r < kVortLoads; ++r) {
    const int i = threadIdx.x + r * kVortThreads;
    if (i < kVortLH * kVortLW) (&S[0][0])[i] = phase_of((double)v[r].re, (double)v[r].im);
  }
  __syncthreads();
  const int lx = threadIdx.x % kVortW;
  const int64_t x = x0 + lx;
  if (x >= f.nu) return;
  const int64_t base = d.psi_off / 5 + pofs;
  for (int k = threadIdx.x / kVortW; k < kVortH; k += kVortThreads / kVortW) {
    const int64_t y = y0 + k;
    if (y >= f.nv) break;
    const int j = k + 1, i = lx + 1;
    const int64_t o = base + y * f.sv + x * f.su;
    if (omega_out) omega_out[o] = curl_of(S[j + 1][i + 1], S[j - 1][i + 1], S[j + 1][i - 1], S[j - 1][i - 1]);
    if (wind_out) wind_out[o] = winding_of(S[j][i], S[j][i + 1], S[j + 1][i + 1], S[j + 1][i]);
  }
}

// ---------------------------------------------------------------------------
// Vorticity and windings of all three plane families of a 3D lattice, fused
// ---------------------------------------------------------------------------
// The planes normal to x (u = y, v = z), to y (u = z, v = x) and to z (u = x,
// v = y) each take the 2D rule above; every output at (x, y, z) needs the phase
// only at offsets in {-1, 0, 1}^3 with at most two non-zero.  A workgroup owns a
// 64 x 16 tile of (x, y) columns and marches over kV3Z consecutive z: the phases
// of the tile and its one-site halo in x and y sit in LDS for four z slices, a
// ring in which slice z+1 overwrites slice z-3, last read two steps earlier,
// before the previous step's barrier, so one barrier per z step suffices.  psi
// of slice z+2 is loaded into registers before the outputs of slice z are
// computed, and turned into phases at the start of the next step.  The phases
// are thus computed 1.16 x (1 + 2 / kV3Z) = 1.31 times per site instead of 3.3
// times, psi is read once instead of once per family, and every store runs
// along x.
constexpr int kV3W = 64, kV3H = 16, kV3Z = 16, kV3Threads = 256;
constexpr int kV3LW = kV3W + 2, kV3LH = kV3H + 2, kV3Slots = 4;
constexpr int kV3Loads = (kV3LW * kV3LH + kV3Threads - 1) / kV3Threads;

template <typename T>
__global__ __launch_bounds__(kV3Threads) void k_vorticity3d(const cx<T>* __restrict__ st, InstDesc d, int m,
                                                           int64_t block0, int64_t cstride,
                                                           double* __restrict__ omega_out,
                                                           int32_t* __restrict__ wind_out) {
#pragma clang fp contract(off)
  __shared__ double P[kV3Slots][kV3LH][kV3LW];
  const int64_t ntx = (d.nx + kV3W - 1) / kV3W, nty = (d.ny + kV3H - 1) / kV3H;
  // the workgroups one XCD runs (every eighth in launch order) take consecutive
  // tiles, so the halo lines shared by x and y neighbours meet in one L2
  int64_t blk = blockIdx.x;
  if (gridDim.x % 8 == 0) blk = (blk % 8) * (gridDim.x / 8) + blk / 8;
  blk += block0;
  const int64_t x0 = (blk % ntx) * kV3W, y0 = ((blk / ntx) % nty) * kV3H, z0 = (blk / (ntx * nty)) * kV3Z;
  const int64_t nxy = (int64_t)d.nx * d.ny;
  const int nzl = (int)((int64_t)d.nz - z0 < kV3Z ? (int64_t)d.nz - z0 : kV3Z);
  const cx<T>* pa = st + d.off + (int64_t)m * d.stride;
  const cx<T>* pb = st + d.off + (int64_t)(5 + m) * d.stride;
  // in-plane offsets of this thread's halo-tile elements, the same for every slice
  int64_t ofs[kV3Loads];
#pragma unroll
  for (int r = 0; r < kV3Loads; ++r) {
    const int i = threadIdx.x + r * kV3Threads;
    const int ly = i / kV3LW, lx = i - ly * kV3LW;
    ofs[r] = i < kV3LW * kV3LH
                 ? (int64_t)wrap_coord(y0 - 1 + ly, d.ny) * d.nx + (int64_t)wrap_coord(x0 - 1 + lx, d.nx)
                 : -1;
  }
  cx<T> v[kV3Loads];
  auto load = [&](int64_t z) {
    const int64_t zo = (int64_t)wrap_coord(z, d.nz) * nxy;
#pragma unroll
    for (int r = 0; r < kV3Loads; ++r)
      if (ofs[r] >= 0) v[r] = pa[zo + ofs[r]] + pb[zo + ofs[r]];
  };
  auto store_phases = [&](int slot) {
#pragma unroll
    for (int r = 0; r < kV3Loads; ++r)
      if (ofs[r] >= 0) (&P[slot][0][0])[threadIdx.x + r * kV3Threads] = phase_of((double)v[r].re, (double)v[r].im);
  };
  // slot of slice z is (z - z0 + 1) mod 4: z0 - 1 in slot 0, z0 in slot 1
  load(z0 - 1);
  store_phases(0);
  load(z0);
  store_phases(1);
  load(z0 + 1);
  const int lane = threadIdx.x % kV3W;
  const int64_t x = x0 + lane;
  const int i = lane + 1;
  const int64_t base = d.psi_off / 5;
  for (int k = 0; k < nzl; ++k) {
    const int sm = k % kV3Slots, s0 = (k + 1) % kV3Slots, sp = (k + 2) % kV3Slots;
    store_phases(sp);
    if (k + 1 < nzl) load(z0 + k + 2);
    __syncthreads();
    if (x < d.nx) {
      const int64_t z = z0 + k;
      for (int r = threadIdx.x / kV3W; r < kV3H; r += kV3Threads / kV3W) {
        const int64_t y = y0 + r;
        if (y >= d.ny) break;
        const int j = r + 1;
        const int64_t o = base + z * nxy + y * d.nx + x;
        const double c = P[s0][j][i];
        if (omega_out) {
          // normal x: u = y, v = z
          omega_out[o] = curl_of(P[sp][j + 1][i], P[sm][j + 1][i], P[sp][j - 1][i], P[sm][j - 1][i]);
          // normal y: u = z, v = x
          omega_out[cstride + o] = curl_of(P[sp][j][i + 1], P[sp][j][i - 1], P[sm][j][i + 1], P[sm][j][i - 1]);
          // normal z: u = x, v = y
          omega_out[2 * cstride + o] =
              curl_of(P[s0][j + 1][i + 1], P[s0][j - 1][i + 1], P[s0][j + 1][i - 1], P[s0][j - 1][i - 1]);
        }
        if (wind_out) {
          wind_out[o] = winding_of(c, P[s0][j + 1][i], P[sp][j + 1][i], P[sp][j][i]);
          wind_out[cstride + o] = winding_of(c, P[sp][j][i], P[sp][j][i + 1], P[s0][j][i + 1]);
          wind_out[2 * cstride + o] = winding_of(c, P[s0][j][i + 1], P[s0][j + 1][i + 1], P[s0][j + 1][i]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Vortex cores: the plaquettes with a non-zero winding, as an ordered list
// ---------------------------------------------------------------------------
// Three launches, no atomics, so the list is in (family, instance, z, y, x)
// order on every run: the non-zero count of every 256-site chunk of every plane
// family (one family in 2D, three in 3D); one workgroup's exclusive scan of the
// counts (the chunks of an instance are consecutive, then the instances, then
// the families); then every chunk writes its cores at its offset, ranked inside
// the chunk by wave ballots.  Workgroup b takes family b / nchunks and chunk
// b % nchunks; family c's windings sit at c * cstride.
__global__ __launch_bounds__(kChunk) void k_core_count(const int32_t* __restrict__ wind, LaunchGeom g,
                                                      int64_t cstride, int64_t* __restrict__ counts) {
  __shared__ int wsum[kChunk / kLanes];
  const int c = blockIdx.x / g.nchunks, b = blockIdx.x - c * g.nchunks;
  const InstDesc d = g.inst[g.chunk2inst[b]];
  const int s = (b - d.chunk_begin) * kChunk + threadIdx.x;
  const bool core = s < d.sites && wind[c * cstride + d.psi_off / 5 + s] != 0;
  const int n = __popcll(__ballot(core));
  if ((threadIdx.x & (kLanes - 1)) == 0) wsum[threadIdx.x / kLanes] = n;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int k = 0; k < kChunk / kLanes; ++k) t += wsum[k];
    counts[blockIdx.x] = t;
  }
}

constexpr int kScanThreads = 1024;

// In place: counts[c] <- sum of counts[0..c), and *total <- the sum of all.
__global__ __launch_bounds__(kScanThreads) void k_core_scan(int64_t* __restrict__ counts, int nchunks,
                                                           int64_t* __restrict__ total) {
  __shared__ int64_t buf[kScanThreads];
  int64_t carry = 0;
  for (int base = 0; base < nchunks; base += kScanThreads) {
    const int i = base + threadIdx.x;
    const int64_t v = i < nchunks ? counts[i] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    // Hillis-Steele inclusive scan over the block
    for (int off = 1; off < kScanThreads; off <<= 1) {
      const int64_t add = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
      __syncthreads();
      buf[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < nchunks) counts[i] = carry + buf[threadIdx.x] - v;
    carry += buf[kScanThreads - 1];
    __syncthreads();   // buf is rewritten by the next block of chunks
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kChunk) void k_core_scatter(const int32_t* __restrict__ wind, LaunchGeom g,
                                                        int ndim, int64_t cstride,
                                                        const int64_t* __restrict__ offsets,
                                                        int32_t* __restrict__ out, int64_t capacity) {
  __shared__ int wsum[kChunk / kLanes];
  const int c = blockIdx.x / g.nchunks, b = blockIdx.x - c * g.nchunks;
  const int inst = g.chunk2inst[b];
  const InstDesc d = g.inst[inst];
  const int s = (b - d.chunk_begin) * kChunk + threadIdx.x;
  const int32_t w = s < d.sites ? wind[c * cstride + d.psi_off / 5 + s] : 0;
  const unsigned long long mask = __ballot(w != 0);
  const int lane = threadIdx.x & (kLanes - 1), wv = threadIdx.x / kLanes;
  if (lane == 0) wsum[wv] = __popcll(mask);
  __syncthreads();
  if (w == 0) return;
  int64_t k = offsets[blockIdx.x] + __popcll(mask & ((1ull << lane) - 1ull));
  for (int j = 0; j < wv; ++j) k += wsum[j];
  if (k >= capacity) return;
  if (ndim == 3) {
    const int nxy = d.nx * d.ny;
    int32_t* e = out + 6 * k;
    e[0] = inst;
    e[1] = c;
    e[2] = s / nxy;
    e[3] = (s % nxy) / d.nx;
    e[4] = s % d.nx;
    e[5] = w;
  } else {
    int32_t* e = out + 4 * k;
    e[0] = inst;
    e[1] = s / d.nx;
    e[2] = s % d.nx;
    e[3] = w;
  }
}

}  // namespace

hipError_t launch_fields(int dtype, const void* state, const LaunchGeom& g, double* n, double* f_par,
                         double* f_perp, double* a00, hipStream_t st) {
  if (g.nchunks == 0) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(k_fields<float>, dim3(g.nchunks), dim3(kChunk), 0, st, (const cx<float>*)state, g, n,
                       f_par, f_perp, a00);
  else
    hipLaunchKernelGGL(k_fields<double>, dim3(g.nchunks), dim3(kChunk), 0, st, (const cx<double>*)state, g,
                       n, f_par, f_perp, a00);
  return hipGetLastError();
}

static int64_t vorticity_blocks(const PlaneFamily& f) {
  return (int64_t)((f.nu + kVortW - 1) / kVortW) * ((f.nv + kVortH - 1) / kVortH) * f.np;
}

static hipError_t launch_family(int dtype, const void* state, const InstDesc& d, const PlaneFamily& f, int m,
                                double* omega, int32_t* winding, hipStream_t st) {
  // pieces of at most 2^22 workgroups keep every launch far below 2^32 work-items
  constexpr int64_t kPiece = int64_t(1) << 22;
  const int64_t nb = vorticity_blocks(f);
  for (int64_t b0 = 0; b0 < nb; b0 += kPiece) {
    const unsigned n = (unsigned)(nb - b0 < kPiece ? nb - b0 : kPiece);
    if (dtype == 0)
      hipLaunchKernelGGL(k_vorticity<float>, dim3(n), dim3(kVortThreads), 0, st, (const cx<float>*)state, d, f,
                         m, b0, omega, winding);
    else
      hipLaunchKernelGGL(k_vorticity<double>, dim3(n), dim3(kVortThreads), 0, st, (const cx<double>*)state, d,
                         f, m, b0, omega, winding);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_vorticity(int dtype, int ndim, const void* state, const InstDesc& d, int m, double* omega,
                            int32_t* winding, int64_t component_stride, hipStream_t st) {
  if (ndim == 2) return launch_family(dtype, state, d, PlaneFamily{d.nx, d.ny, 1, 1, d.nx, 0}, m, omega, winding, st);
  // 3D: the families normal to x, y and z, one after the other in the outputs, in one pass
  constexpr int64_t kPiece = int64_t(1) << 22;
  const int64_t nb = (int64_t)((d.nx + kV3W - 1) / kV3W) * ((d.ny + kV3H - 1) / kV3H) * ((d.nz + kV3Z - 1) / kV3Z);
  for (int64_t b0 = 0; b0 < nb; b0 += kPiece) {
    const unsigned n = (unsigned)(nb - b0 < kPiece ? nb - b0 : kPiece);
    if (dtype == 0)
      hipLaunchKernelGGL(k_vorticity3d<float>, dim3(n), dim3(kV3Threads), 0, st, (const cx<float>*)state, d, m, b0,
                         component_stride, omega, winding);
    else
      hipLaunchKernelGGL(k_vorticity3d<double>, dim3(n), dim3(kV3Threads), 0, st, (const cx<double>*)state, d, m,
                         b0, component_stride, omega, winding);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_vortex_cores(const int32_t* winding, const LaunchGeom& g, int ndim, int64_t component_stride,
                               int64_t* counts, int32_t* out, int64_t capacity, int64_t* total, hipStream_t st) {
  if (g.nchunks == 0) return hipSuccess;
  const int nblocks = (ndim == 3 ? 3 : 1) * g.nchunks;
  hipLaunchKernelGGL(k_core_count, dim3(nblocks), dim3(kChunk), 0, st, winding, g, component_stride, counts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_core_scan, dim3(1), dim3(kScanThreads), 0, st, counts, nblocks, total);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_core_scatter, dim3(nblocks), dim3(kChunk), 0, st, winding, g, ndim, component_stride, counts,
                     out, capacity);
  return hipGetLastError();
}

}  // namespace qlg
