// Kernels of the reverse-mode (adjoint) QLG step.
//
// The adjoint walks each step's substeps backwards.  The kinetic factors are
// linear and unitary, so their pull-back is the exact inverse I'^H = C^H S C^H S^T
// applied to the cotangent (no stored state).  The self-interaction is
// nonlinear: its pull-back (qlg_vjp.hpp, FP64) needs the substep's input
// state, which a chain of per-substep kernels regenerates from the segment's
// checkpoint (the per-site formulas of the fused forward kernels; the compiler
// may contract them into FMAs differently, so the regenerated FP32 states can
// differ from the forward's in the last bit).
//
// All kernels are one thread per site over 256-site chunks of each instance.

#include <algorithm>

#include "qlg_adjoint_kernels.hpp"
#include "qlg_math.hpp"
#include "qlg_vjp.hpp"

namespace qlg {

namespace {

struct Site {
  InstDesc d;
  int c;            // the 256-site chunk this workgroup owns
  int s, x, y, z;
  bool ok;
};

// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each with its own L2.
// Consecutive chunks (a row and the rows next to it, whose cotangents and states the kinetic
// pull-back and the chain's I' read again) are given to one XCD, so that those re-reads hit
// its L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int chunk_of_block(int b, int nblocks) {
  const int x = b % kXcds, l = b / kXcds;
  const int per = nblocks / kXcds, extra = nblocks % kXcds;
  return x * per + (x < extra ? x : extra) + l;
}

// This thread's site in chunk c (thread t of the workgroup takes site t of the chunk).
__device__ __forceinline__ Site site_of_chunk(const LaunchGeom& g, int c) {
  Site r;
  r.c = c;
  r.d = g.inst[g.chunk2inst[c]];
  r.s = (c - r.d.chunk_begin) * kChunk + threadIdx.x;
  r.ok = r.s < r.d.sites;
  r.x = r.ok ? r.s % r.d.nx : 0;
  r.y = r.ok ? (r.s / r.d.nx) % r.d.ny : 0;
  r.z = r.ok ? r.s / (r.d.nx * r.d.ny) : 0;
  return r;
}

__device__ __forceinline__ Site site_here(const LaunchGeom& g) {
  return site_of_chunk(g, chunk_of_block(blockIdx.x, gridDim.x));
}

// site index of the neighbour at offset dir (+1 / -1) along axis (0 = x, 1 = y, 2 = z), periodic
__device__ __forceinline__ int neighbour(const Site& r, int axis, int dir) {
  // one branch per axis: selecting the extent by a run-time axis index puts them on the stack
  if (axis == 0) {
    int x = r.x + dir;
    x = x < 0 ? x + r.d.nx : (x >= r.d.nx ? x - r.d.nx : x);
    return r.s - r.x + x;
  }
  if (axis == 1) {
    int y = r.y + dir;
    y = y < 0 ? y + r.d.ny : (y >= r.d.ny ? y - r.d.ny : y);
    return r.s + (y - r.y) * r.d.nx;
  }
  int z = r.z + dir;
  z = z < 0 ? z + r.d.nz : (z >= r.d.nz ? z - r.d.nz : z);
  return r.s + (z - r.z) * r.d.nx * r.d.ny;
}

template <typename T, typename S>
__device__ __forceinline__ void load_site(const cx<T>* __restrict__ st, const InstDesc& d, int s,
                                          cx<S> (&a)[5], cx<S> (&b)[5]) {
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const cx<T> va = st[d.off + m * d.stride + s];
    const cx<T> vb = st[d.off + (5 + m) * d.stride + s];
    a[m] = cx<S>{(S)va.re, (S)va.im};
    b[m] = cx<S>{(S)vb.re, (S)vb.im};
  }
}

template <typename T>
__device__ __forceinline__ void store_site(cx<T>* __restrict__ st, const InstDesc& d, int s, const cx<T> (&a)[5],
                                           const cx<T> (&b)[5]) {
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    st[d.off + m * d.stride + s] = a[m];
    st[d.off + (5 + m) * d.stride + s] = b[m];
  }
}

// The same, with the non-temporal hint: for the recorded self-interaction
// inputs, written once per segment recompute and read back once, by the
// reverse sweep, so they need not displace lines the recompute still reads.
template <typename T>
__device__ __forceinline__ void store_site_nt(cx<T>* __restrict__ st, const InstDesc& d, int s, const cx<T> (&a)[5],
                                              const cx<T> (&b)[5]) {
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    cx<T>* pa = st + d.off + m * d.stride + s;
    cx<T>* pb = st + d.off + (5 + m) * d.stride + s;
    __builtin_nontemporal_store(a[m].re, &pa->re);
    __builtin_nontemporal_store(a[m].im, &pa->im);
    __builtin_nontemporal_store(b[m].re, &pb->re);
    __builtin_nontemporal_store(b[m].im, &pb->im);
  }
}
template <typename T, typename S>
__device__ __forceinline__ void load_site_nt(const cx<T>* __restrict__ st, const InstDesc& d, int s,
                                             cx<S> (&a)[5], cx<S> (&b)[5]) {
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const cx<T>* pa = st + d.off + m * d.stride + s;
    const cx<T>* pb = st + d.off + (5 + m) * d.stride + s;
    a[m] = cx<S>{(S)__builtin_nontemporal_load(&pa->re), (S)__builtin_nontemporal_load(&pa->im)};
    b[m] = cx<S>{(S)__builtin_nontemporal_load(&pb->re), (S)__builtin_nontemporal_load(&pb->im)};
  }
}

// C^H without its factor 1/2:  2 a' = (a + b) + i (a - b),  2 b' = (a + b) - i (a - b)
__device__ __forceinline__ void collide2_adj(cx<double> (&a)[5], cx<double> (&b)[5]) {
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const double sr = a[m].re + b[m].re, si = a[m].im + b[m].im;
    const double dr = a[m].re - b[m].re, di = a[m].im - b[m].im;
    a[m] = cx<double>{sr - di, si + dr};
    b[m] = cx<double>{sr + di, si - dr};
  }
}

// Moves of a double by one lane across the whole wavefront (DPP wave_shl:1 / wave_shr:1);
// the end lane, a halo lane here, reads 0.
template <int Ctrl>
__device__ __forceinline__ double lane_move(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, Ctrl, 0xF, 0xF, true);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), Ctrl, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
constexpr int kFromNextLane = 0x130;   // lane i reads lane i + 1
constexpr int kFromPrevLane = 0x138;   // lane i reads lane i - 1
template <int Ctrl>
__device__ __forceinline__ float lane_move(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), Ctrl, 0xF, 0xF, true));
}
template <int Ctrl, typename T>
__device__ __forceinline__ cx<T> lane_move(cx<T> v) {
  return cx<T>{lane_move<Ctrl>(v.re), lane_move<Ctrl>(v.im)};
}

// I'_{x,q} with x along the lanes, in the operation order of iprime_site: C, q from x + 1, C,
// q from x - 1, and its exact 1/4.  Q = 1: qubit b moves; Q = 0: qubit a.
template <int Q, typename T>
__device__ __forceinline__ void iprime_lanes(cx<T> (&a)[5], cx<T> (&b)[5]) {
  collide2(a, b);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    if (Q) b[m] = lane_move<kFromNextLane>(b[m]);
    else   a[m] = lane_move<kFromNextLane>(a[m]);
  }
  collide2(a, b);
  scale_quarter(a, b);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    if (Q) b[m] = lane_move<kFromPrevLane>(b[m]);
    else   a[m] = lane_move<kFromPrevLane>(a[m]);
  }
}

// lambda <- I'^H_{x,q} lambda with x along the lanes: q from x + 1, C^H, q from x - 1, C^H, 1/4
// (the order of iprime_adj_site).  Q = 1: qubit b moves; Q = 0: qubit a.
template <int Q>
__device__ __forceinline__ void iprime_adj_lanes(cx<double> (&a)[5], cx<double> (&b)[5]) {
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    if (Q) b[m] = lane_move<kFromNextLane>(b[m]);
    else   a[m] = lane_move<kFromNextLane>(a[m]);
  }
  collide2_adj(a, b);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    if (Q) b[m] = lane_move<kFromPrevLane>(b[m]);
    else   a[m] = lane_move<kFromPrevLane>(a[m]);
  }
  collide2_adj(a, b);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    a[m] = 0.25 * a[m];
    b[m] = 0.25 * b[m];
  }
}

}  // namespace

// (I' in)(x) for I'_{axis,q} = S_q C S_q^T C, from `in` at x-1, x, x+1, with the fused
// kernels' operation order: c = C(in) at x-1, x, x+1;  t(y) = (c.nonq(y), c.q(y+1));
// m(y) = C t(y) (two unscaled collides and an exact 1/4);  out.nonq(x) = m(x).nonq,
// out.q(x) = m(x-1).q.
template <typename T>
__device__ __forceinline__ void iprime_site(const cx<T>* __restrict__ in, const Site& r, int axis, int qb,
                                            cx<T> (&oa)[5], cx<T> (&ob)[5]) {
  const int sm = neighbour(r, axis, -1), sp = neighbour(r, axis, +1);
  cx<T> a0[5], b0[5], a1[5], b1[5], a2[5], b2[5];   // x-1, x, x+1
  load_site(in, r.d, sm, a0, b0);
  load_site(in, r.d, r.s, a1, b1);
  load_site(in, r.d, sp, a2, b2);
  collide2(a0, b0);
  collide2(a1, b1);
  collide2(a2, b2);
  cx<T> ta[5], tb[5], ua[5], ub[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    // t(x) = (nonq of c(x), q of c(x+1));  t(x-1) = (nonq of c(x-1), q of c(x))
    ta[m] = sel(qb != 0, a1[m], a2[m]);
    tb[m] = sel(qb != 0, b2[m], b1[m]);
    ua[m] = sel(qb != 0, a0[m], a1[m]);
    ub[m] = sel(qb != 0, b1[m], b0[m]);
  }
  collide2(ta, tb);
  scale_quarter(ta, tb);
  collide2(ua, ub);
  scale_quarter(ua, ub);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    oa[m] = sel(qb != 0, ta[m], ua[m]);   // moving qubit from m(x-1), the other from m(x)
    ob[m] = sel(qb != 0, ub[m], tb[m]);
  }
}

// One link of the recorded forward chain that regenerates a checkpoint segment:
//   z = I'_{axis,q}(in) at this site (z = in when axis < 0),  rec <- z (when rec is set),
//   out <- U(z) (out <- z when !with_u).
// Successive links walk the substeps "U_k then I'_k" of consecutive steps as
// "I'_{k-1} then U_k", so every input z of a self-interaction is written once.
// theta (V + mu) at a site, for a context with an external or chemical potential
__device__ __forceinline__ double ext_here(const Site& r, const double* pot, double mu, double theta) {
  return theta * ((pot ? pot[r.d.psi_off / 5 + r.s] : 0.0) + mu);
}

template <typename T>
__global__ __launch_bounds__(kChunk) void k_chain(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                 cx<T>* __restrict__ rec, LaunchGeom g, int axis, int qb,
                                                 int with_u, Angles<T> ang, const double* __restrict__ pot,
                                                 double mu, double theta) {
  const Site r = site_here(g);
  if (!r.ok) return;
  cx<T> a[5], b[5];
  if (axis >= 0) iprime_site(in, r, axis, qb, a, b);
  else load_site(in, r.d, r.s, a, b);
  if (rec) store_site_nt(rec, r.d, r.s, a, b);
  if (with_u) {
    // the same per-site angle as the fused forward kernels: T(theta) T(V + mu)
    if (pot || mu != 0.0) potential<T, true>(a, b, ang, T(theta) * T((pot ? pot[r.d.psi_off / 5 + r.s] : 0.0) + mu));
    else potential(a, b, ang);
  }
  store_site(out, r.d, r.s, a, b);
}

// (I'^H lambda)(x) = (C^H S_q C^H S_q^T lambda)(x) (FP64) from lambda at x-1, x, x+1:
//   w(y) = C^H(lambda.nonq(y), lambda.q(y+1));  out(x) = C^H(w(x).nonq, w(x-1).q).
__device__ __forceinline__ void iprime_adj_site(const cx<double>* __restrict__ in, const Site& r, int axis, int qb,
                                                cx<double> (&oa)[5], cx<double> (&ob)[5]) {
  const int sm = neighbour(r, axis, -1), sp = neighbour(r, axis, +1);
  cx<double> a0[5], b0[5], a1[5], b1[5], a2[5], b2[5];
  load_site(in, r.d, sm, a0, b0);
  load_site(in, r.d, r.s, a1, b1);
  load_site(in, r.d, sp, a2, b2);
  cx<double> wa[5], wb[5], va[5], vb[5];   // w(x), w(x-1)
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    wa[m] = sel(qb != 0, a1[m], a2[m]);
    wb[m] = sel(qb != 0, b2[m], b1[m]);
    va[m] = sel(qb != 0, a0[m], a1[m]);
    vb[m] = sel(qb != 0, b1[m], b0[m]);
  }
  collide2_adj(wa, wb);
  collide2_adj(va, vb);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    oa[m] = sel(qb != 0, wa[m], va[m]);
    ob[m] = sel(qb != 0, vb[m], wb[m]);
  }
  collide2_adj(oa, ob);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    oa[m] = 0.25 * oa[m];
    ob[m] = 0.25 * ob[m];
  }
}

// lambda <- I'^H lambda, out of place.
__global__ __launch_bounds__(kChunk) void k_sub_iprime_adj(const cx<double>* __restrict__ in,
                                                          cx<double>* __restrict__ out, LaunchGeom g, int axis,
                                                          int qb) {
  const Site r = site_here(g);
  if (!r.ok) return;
  cx<double> oa[5], ob[5];
  iprime_adj_site(in, r, axis, qb, oa, ob);
  store_site(out, r.d, r.s, oa, ob);
}

// Block sum of three doubles into dst[0..2] (fixed order).
__device__ __forceinline__ void block_sum3(double v0, double v1, double v2, double* __restrict__ dst) {
  __shared__ double red[3][kChunk / kLanes];
  const int lane = threadIdx.x & (kLanes - 1), wv = threadIdx.x >> 6;
  double v[3] = {v0, v1, v2};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double s = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, kLanes);
    if (lane == 0) red[k][wv] = s;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kChunk / kLanes; ++j) s += red[threadIdx.x][j];
    dst[threadIdx.x] = s;
  }
}

// lambda <- (dU)^H lambda at the substep input z (FP64 Jacobian); dg partials per chunk.
template <typename T>
__global__ __launch_bounds__(kChunk) void k_sub_vjp(const cx<T>* __restrict__ z, cx<double>* __restrict__ lam,
                                                   LaunchGeom g, double theta, double g0, double g1, double g2,
                                                   const double* __restrict__ pot, double mu,
                                                   double* __restrict__ part) {
  const Site r = site_here(g);
  double dg[3] = {0.0, 0.0, 0.0};
  if (r.ok) {
    cx<double> a[5], b[5], la[5], lb[5];
    load_site_nt(z, r.d, r.s, a, b);
    load_site(lam, r.d, r.s, la, lb);
    potential_vjp(a, b, la, lb, theta, g0, g1, g2, dg, ext_here(r, pot, mu, theta));
    store_site(lam, r.d, r.s, la, lb);
  }
  block_sum3(dg[0], dg[1], dg[2], part + 3 * (int64_t)r.c);
}

// One adjoint substep of the interleaved split, fused: lambda_out = (dU)^H I'^H lambda_in,
// the kinetic pull-back recomputed per site from lambda_in at x-1, x, x+1 along `axis`,
// then the FP64 self-interaction VJP at the substep input z; dg partials per wavefront.
// Workgroups of one wavefront (a quarter of a chunk): a wavefront that finishes frees its
// SIMD slot for the next at once, so the two wavefronts of a SIMD drift apart and one loads
// while the other computes.  (Workgroups of a whole chunk, summed in LDS behind a barrier,
// started and ended four wavefronts together, which kept the loads and the arithmetic of a
// SIMD's wavefronts in step.)
template <typename T>
__global__ __launch_bounds__(kLanes) void k_sub_adj(const cx<T>* __restrict__ z,
                                                   const cx<double>* __restrict__ lin,
                                                   cx<double>* __restrict__ lout, LaunchGeom g, int axis, int qb,
                                                   double theta, double g0, double g1, double g2,
                                                   const double* __restrict__ pot, double mu,
                                                   double* __restrict__ part) {
  constexpr int kWaves = kChunk / kLanes;
  // wavefront unit u: quarter u % 4 of chunk u / 4, units of one XCD consecutive
  const int u = chunk_of_block(blockIdx.x, gridDim.x);
  Site r = site_of_chunk(g, u / kWaves);
  r.s += (u % kWaves) * kLanes;   // site_of_chunk counts threadIdx.x from the chunk's start
  r.ok = r.s < r.d.sites;
  r.x = r.ok ? r.s % r.d.nx : 0;
  r.y = r.ok ? (r.s / r.d.nx) % r.d.ny : 0;
  r.z = r.ok ? r.s / (r.d.nx * r.d.ny) : 0;
  double dg[3] = {0.0, 0.0, 0.0};
  if (r.ok) {
    cx<double> la[5], lb[5];
    iprime_adj_site(lin, r, axis, qb, la, lb);
    cx<double> a[5], b[5];
    load_site_nt(z, r.d, r.s, a, b);
    potential_vjp(a, b, la, lb, theta, g0, g1, g2, dg, ext_here(r, pot, mu, theta));
    store_site(lout, r.d, r.s, la, lb);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dg[k] += __shfl_xor(dg[k], o, kLanes);
  }
  if (threadIdx.x == 0) {
    part[3 * (int64_t)u] = dg[0];
    part[3 * (int64_t)u + 1] = dg[1];
    part[3 * (int64_t)u + 2] = dg[2];
  }
}

// Buffer-resource stores (a lane whose offset lies beyond the record count stores nothing), so
// that every path through a loop issues the same memory instructions and the compiler's waits
// for loads issued ahead stay exact.
constexpr int kBufWord3 = 0x00020000;   // resource word 3 on gfx9: 32-bit data format, no swizzle
constexpr uint32_t kOffNone = 0x80000000u;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufWord3);
}

// A wavefront tile of the fused x kernels: 56 columns of one row of one instance plus 4 halo
// columns on each side.  The instance is the last i with xpre[i] <= w; the tables are read
// through the constant address space (scalar loads, not ordered behind vector memory).
struct X4Tile {
  InstDesc d;
  int row;   // row of the instance (y + ny z)
  int s;     // this lane's site (periodic column)
  int x;     // this lane's column before the wrap
  bool own;  // one of the 56 columns this tile writes
};
__device__ __forceinline__ X4Tile x4_tile(const LaunchGeom& g, const int* xpre_g, int w, int lane) {
  typedef const __attribute__((address_space(4))) int32_t* CInt;
  const CInt xpre = (CInt)xpre_g;
  int lo = 0, hi = g.nbatch;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (xpre[mid] <= w) lo = mid;
    else hi = mid;
  }
  static_assert(sizeof(InstDesc) % 4 == 0, "InstDesc is read as 32-bit words");
  constexpr int kWords = (int)(sizeof(InstDesc) / 4);
  const CInt words = (CInt)g.inst + kWords * lo;
  int32_t buf[kWords];
#pragma unroll
  for (int i = 0; i < kWords; ++i) buf[i] = words[i];
  X4Tile r;
  __builtin_memcpy(&r.d, buf, sizeof(InstDesc));
  const int t = w - xpre[lo];
  const int ntx = (r.d.nx + kValid2D - 1) / kValid2D;
  const int tx = t % ntx;
  r.row = t / ntx;
  r.x = tx * kValid2D - kHalo2D + lane;
  const int xw = r.x < 0 ? r.x + r.d.nx * ((-r.x + r.d.nx - 1) / r.d.nx) : r.x % r.d.nx;
  r.own = lane >= kHalo2D && lane < kLanes - kHalo2D && r.x < r.d.nx;
  r.s = r.row * r.d.nx + xw;
  return r;
}

// The four adjoint substeps along x of a step, fused: for k = k0 + 3, ..., k0 (qubits a, a, b, b),
//   lambda <- (dU_k)^H I'^H_{x,q_k} lambda  at the recorded inputs z_k.
// A tile is 56 columns of one row (x tiles of each row, rows of each instance in order,
// instances by the prefix table xpre) plus 4 halo columns on each side: each I'^H reaches one
// site, so after the four substeps the middle 56 lanes hold the cotangent of their sites, read
// and written once instead of once per substep.  The x shifts are lane moves.  Only the 56 owned
// lanes add to the dg partial of the tile (part[3 w + 0..2]).
// One wavefront per SIMD (its registers, 256 + about 130 accumulation registers, do not fit the
// 256 of two waves without spilling to scratch, which measured 1.5x slower), persistent: a
// wavefront walks tiles of its XCD's contiguous range, and during a tile's last substep it loads
// the next tile's cotangent, potential and first record, whose latency a wavefront alone on its
// SIMD would otherwise wait out at the start of every tile.
template <typename T>
__global__ __launch_bounds__(kChunk) void k_adj_x4(const cx<T>* __restrict__ z3, const cx<T>* __restrict__ z2,
                                                  const cx<T>* __restrict__ z1, const cx<T>* __restrict__ z0,
                                                  const cx<double>* __restrict__ lin, cx<double>* __restrict__ lout,
                                                  LaunchGeom g, const int* __restrict__ xpre, int nwaves,
                                                  double theta, double g0, double g1, double g2,
                                                  const double* __restrict__ pot, double mu,
                                                  double* __restrict__ part) {
  constexpr int kWaves = kChunk / kLanes;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & (kLanes - 1);
  // tiles [c0, c1) of this workgroup's XCD, taken with the stride of the XCD's wavefront count
  // (a grid of fewer than 8 workgroups: each workgroup a group of its own)
  const int nb = gridDim.x, ng = nb < kXcds ? nb : kXcds;
  const int xcd = blockIdx.x % ng, lb = blockIdx.x / ng;
  const int stride = (nb / ng + (xcd < nb % ng ? 1 : 0)) * kWaves;
  const int per = nwaves / ng, extra = nwaves % ng;
  const int c0 = xcd * per + (xcd < extra ? xcd : extra);
  const int c1 = c0 + per + (xcd < extra ? 1 : 0);
  int w = c0 + lb * kWaves + wv;
  if (w >= c1) return;   // wavefront-uniform; no workgroup-level synchronisation below
  // the potential's phase at a site: a resource of size 0 without a potential reads 0
  auto ext_at = [&](const X4Tile& t) __attribute__((always_inline)) {
    const __amdgpu_buffer_rsrc_t pr = buf_rsrc(pot ? pot + t.d.psi_off / 5 : nullptr,
                                               pot ? (uint32_t)t.d.sites * 8u : 0u);
    const double v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(pr, t.s * 8, 0, 0));
    return theta * (v + mu);
  };
  // the records of substeps k0 + 2, k0 + 1, k0 as a pointer formed by arithmetic (a select
  // between three pointers in a loop is otherwise made a table in private memory)
  auto zrec = [&](int i) __attribute__((always_inline)) {
    const uintptr_t p = (uintptr_t)z2 * (uintptr_t)(i == 0) + (uintptr_t)z1 * (uintptr_t)(i == 1) +
                        (uintptr_t)z0 * (uintptr_t)(i == 2);
    return (const cx<T>*)p;
  };
  cx<double> nla[5], nlb[5];
  cx<T> na[5], nb5[5];
  double next_ext;
  {
    const X4Tile t0 = x4_tile(g, xpre, w, lane);
    load_site(lin, t0.d, t0.s, nla, nlb);
    next_ext = ext_at(t0);
    load_site_nt(z3, t0.d, t0.s, na, nb5);
  }
  for (;;) {
    const X4Tile cur = x4_tile(g, xpre, w, lane);
    cx<double> la[5], lb5[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      la[m] = nla[m];
      lb5[m] = nlb[m];
    }
    const double ext = next_ext;
    double dg[3] = {0.0, 0.0, 0.0};
    // substeps k0 + 3, k0 + 2 (qubit a), k0 + 1 (qubit b), each at the record in na, nb5 and
    // loading the next one
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
      cx<double> a[5], b[5];
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        a[m] = cx<double>{(double)na[m].re, (double)na[m].im};
        b[m] = cx<double>{(double)nb5[m].re, (double)nb5[m].im};
      }
      load_site_nt(zrec(i), cur.d, cur.s, na, nb5);
      if (i < 2) iprime_adj_lanes<0>(la, lb5);
      else iprime_adj_lanes<1>(la, lb5);
      double dgl[3] = {0.0, 0.0, 0.0};
      potential_vjp<true>(a, b, la, lb5, theta, g0, g1, g2, dgl, ext);
#pragma unroll
      for (int k = 0; k < 3; ++k) dg[k] += cur.own ? dgl[k] : 0.0;
    }
    // substep k0 (qubit b), with the next tile's cotangent, potential and first record loaded
    // first (the last tile loads its own again: nothing writes lin, pot or the records)
    const int wn = w + stride;
    const bool more = wn < c1;
    {
      cx<double> a[5], b[5];
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        a[m] = cx<double>{(double)na[m].re, (double)na[m].im};
        b[m] = cx<double>{(double)nb5[m].re, (double)nb5[m].im};
      }
      const X4Tile nt = x4_tile(g, xpre, more ? wn : w, lane);
      load_site(lin, nt.d, nt.s, nla, nlb);
      next_ext = ext_at(nt);
      load_site_nt(z3, nt.d, nt.s, na, nb5);
      iprime_adj_lanes<1>(la, lb5);
      double dgl[3] = {0.0, 0.0, 0.0};
      potential_vjp<true>(a, b, la, lb5, theta, g0, g1, g2, dgl, ext);
#pragma unroll
      for (int k = 0; k < 3; ++k) dg[k] += cur.own ? dgl[k] : 0.0;
    }
    // the owned columns' cotangents: one row of each plane, lanes outside it drop their stores
    const uint32_t off = cur.own ? (uint32_t)cur.x * 16u : kOffNone;
    const uint32_t rb = (uint32_t)cur.d.nx * 16u;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const cx<double>* pa = lout + cur.d.off + m * cur.d.stride + (int64_t)cur.row * cur.d.nx;
      const cx<double>* pb = lout + cur.d.off + (5 + m) * cur.d.stride + (int64_t)cur.row * cur.d.nx;
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, la[m]), buf_rsrc(pa, rb), (int)off, 0, 0);
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, lb5[m]), buf_rsrc(pb, rb), (int)off, 0, 0);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) dg[k] += __shfl_xor(dg[k], o, kLanes);
    }
    // lanes 0, 1, 2 store dg[0], dg[1], dg[2] of the tile
    const double mine = lane == 0 ? dg[0] : lane == 1 ? dg[1] : dg[2];
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, mine), buf_rsrc(part + 3 * (int64_t)w, 24u),
                                          (int)(lane < 3 ? (uint32_t)lane * 8u : kOffNone), 0, 0);
    if (!more) break;
    w = wn;
  }
}

// The links of the recorded forward chain that apply x kinetic factors, fused: for the links
// (j, nsub - 3), (j, nsub - 2), (j, nsub - 1) and, when r3 is set, (j + 1, 0),
//   z <- I'_{x,q}(y) (q = b, b, a, a),  r_i <- z,  y <- U(z),
// on the tiles of k_adj_x4 (56 columns of one row plus 4 halo columns on each side, the x
// shifts as lane moves): the state is read and written once for the four links.  Only the
// owned lanes store their records and the output.
template <typename T>
__global__ __launch_bounds__(kChunk) void k_chain_x4(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                    cx<T>* __restrict__ r0, cx<T>* __restrict__ r1,
                                                    cx<T>* __restrict__ r2, cx<T>* __restrict__ r3,
                                                    LaunchGeom g, const int* __restrict__ xpre, int nwaves,
                                                    Angles<T> ang, const double* __restrict__ pot, double mu,
                                                    double theta) {
  constexpr int kWaves = kChunk / kLanes;
  const int w = chunk_of_block(blockIdx.x, gridDim.x) * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (w >= nwaves) return;
  const int lane = threadIdx.x & (kLanes - 1);
  int lo = 0, hi = g.nbatch;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (xpre[mid] <= w) lo = mid;
    else hi = mid;
  }
  const InstDesc d = g.inst[lo];
  const int t = w - xpre[lo];
  const int ntx = (d.nx + kValid2D - 1) / kValid2D;
  const int tx = t % ntx, row = t / ntx;
  const int x = tx * kValid2D - kHalo2D + lane;
  const int xw = x < 0 ? x + d.nx * ((-x + d.nx - 1) / d.nx) : x % d.nx;
  const bool own = lane >= kHalo2D && lane < kLanes - kHalo2D && x < d.nx;
  const int s = row * d.nx + xw;
  cx<T> a[5], b[5];
  load_site(in, d, s, a, b);
  const bool ext = pot || mu != 0.0;
  const T e = T(theta) * T((pot ? pot[d.psi_off / 5 + s] : 0.0) + mu);
  auto link = [&](cx<T>* __restrict__ rec) {
    if (own) store_site_nt(rec, d, s, a, b);
    if (ext) potential<T, true>(a, b, ang, e);
    else potential(a, b, ang);
  };
  iprime_lanes<1>(a, b);
  link(r0);
  iprime_lanes<1>(a, b);
  link(r1);
  iprime_lanes<0>(a, b);
  link(r2);
  if (r3) {
    iprime_lanes<0>(a, b);
    link(r3);
  }
  if (own) store_site(out, d, s, a, b);
}

// xpre[i] = wavefronts of k_adj_x4 before instance i (xpre[nbatch] = all of them).
__global__ void k_x4_prefix(LaunchGeom g, int* __restrict__ xpre) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int acc = 0;
  for (int i = 0; i < g.nbatch; ++i) {
    xpre[i] = acc;
    const InstDesc d = g.inst[i];
    acc += (d.nx + kValid2D - 1) / kValid2D * d.ny * d.nz;
  }
  xpre[g.nbatch] = acc;
}

// acc[0..2] += sum over chunks of part (single block, fixed order).  Unrolling
// issues the loads of eight chunks ahead of their additions; each thread still
// adds its chunks in increasing order.
// One workgroup of 1024 threads: thread t sums the partials t, t + 1024, ... (a serial chain of
// a few dozen loads each), then the 16 wavefront sums are added in order.
constexpr int kDgThreads = 1024;
__global__ __launch_bounds__(kDgThreads) void k_dg_accumulate(const double* __restrict__ part, int nparts,
                                                            double* __restrict__ acc) {
  constexpr int kW = kDgThreads / kLanes;
  __shared__ double red[3][kW];
  const int lane = threadIdx.x & (kLanes - 1), wv = threadIdx.x >> 6;
  double v[3] = {0.0, 0.0, 0.0};
#pragma unroll 8
  for (int c = threadIdx.x; c < nparts; c += kDgThreads) {
    v[0] += part[3 * c];
    v[1] += part[3 * c + 1];
    v[2] += part[3 * c + 2];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, kLanes);
    if (lane == 0) red[k][wv] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < kW; ++j) t += red[threadIdx.x][j];
    acc[threadIdx.x] += t;
  }
}

// First stage of launch_dg_reduce: workgroup b sums the partials of its contiguous range
// [b n / G, (b + 1) n / G) (thread t: entries t, t + 256, ... of the range; then the four
// wavefront sums in order) into red[b][0..2].
__global__ __launch_bounds__(kChunk) void k_dg_blocks(const double* __restrict__ part, int64_t n,
                                                     double* __restrict__ red) {
  const int64_t G = gridDim.x;
  const int64_t lo = n * blockIdx.x / G, hi = n * (blockIdx.x + 1) / G;
  double v[3] = {0.0, 0.0, 0.0};
#pragma unroll 8
  for (int64_t c = lo + threadIdx.x; c < hi; c += kChunk) {
    v[0] += part[3 * c];
    v[1] += part[3 * c + 1];
    v[2] += part[3 * c + 2];
  }
  block_sum3(v[0], v[1], v[2], red + 3 * (int64_t)blockIdx.x);
}

// Energy objective: lambda_a = lambda_b = 2 dE/dpsi* written in the canonical
// complex128 qubits layout; per chunk partials part[6c + 0..3] of
// eps^d x (E density, n^2/2, |F|^2/2, |sigma|^2/10).
template <typename T>
__global__ __launch_bounds__(kChunk) void k_energy_grad(const cx<T>* __restrict__ st, cx<double>* __restrict__ lam,
                                                       LaunchGeom g, int ndim, double eps, double g0,
                                                       double g1, double g2, const double* __restrict__ pot,
                                                       double mu, double* __restrict__ part) {
  const Site r = site_here(g);
  double e = 0.0, en = 0.0, ef = 0.0, es = 0.0;
  if (r.ok) {
    const double meas = ndim == 1 ? eps : ndim == 2 ? eps * eps : eps * eps * eps;
    const double ie2 = 1.0 / (eps * eps);
    cx<double> a[5], b[5], p[5], lap[5];
    load_site(st, r.d, r.s, a, b);
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      p[m] = a[m] + b[m];
      lap[m] = cx<double>{0.0, 0.0};
    }
    double ekin = 0.0;
    for (int axis = 0; axis < ndim; ++axis) {
      cx<double> pa[5], pb[5], ma[5], mb[5];
      load_site(st, r.d, neighbour(r, axis, +1), pa, pb);
      load_site(st, r.d, neighbour(r, axis, -1), ma, mb);
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const cx<double> pp = pa[m] + pb[m], pm = ma[m] + mb[m];
        const cx<double> df = pp - p[m];
        ekin += df.re * df.re + df.im * df.im;
        lap[m] = lap[m] + (2.0 * p[m] - pp - pm);
      }
    }
    // H_loc psi = g0 n psi + g1 (F.f) psi + (g2/5) sigma S psi*
    double q[5], n = 0.0;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      q[m] = p[m].re * p[m].re + p[m].im * p[m].im;
      n += q[m];
    }
    const double Fz = 2.0 * (q[0] - q[4]) + (q[1] - q[3]);
    const cx<double> f1 = cmulc(p[0], p[1]) + cmulc(p[3], p[4]);
    const cx<double> f2 = cmulc(p[1], p[2]) + cmulc(p[2], p[3]);
    const double Fx = 2.0 * f1.re + Consts::r6 * f2.re, Fy = 2.0 * f1.im + Consts::r6 * f2.im;
    const cx<double> sig = 2.0 * (p[0] * p[4]) - 2.0 * (p[1] * p[3]) + p[2] * p[2];
    const double cf[4] = {2.0, Consts::r6, Consts::r6, 2.0};
    cx<double> fp[5] = {}, fm[5] = {};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      fp[i] = cf[i] * p[i + 1];
      fm[i + 1] = cf[i] * p[i];
    }
    const cx<double> cpl{0.5 * Fx, -0.5 * Fy}, cmi{0.5 * Fx, 0.5 * Fy};
    const double vmu = ext_here(r, pot, mu, 1.0);   // V + mu at this site (0 without a potential)
    cx<double> Sp[5];
    {
      cx<double> pc[5];
#pragma unroll
      for (int m = 0; m < 5; ++m) pc[m] = conj(p[m]);
      Sp[0] = pc[4]; Sp[1] = -1.0 * pc[3]; Sp[2] = pc[2]; Sp[3] = -1.0 * pc[1]; Sp[4] = pc[0];
    }
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      cx<double> h = (g0 * n + vmu) * p[m] + g1 * ((Fz * (2 - m)) * p[m] + cpl * fp[m] + cmi * fm[m]);
      h = h + (g2 / 5.0) * (sig * Sp[m]);
      const cx<double> l = (2.0 * meas) * (ie2 * lap[m] + h);
      const int64_t o = r.d.qb_off + (int64_t)m * r.d.sites + r.s;
      lam[o] = l;
      lam[o + 5 * (int64_t)r.d.sites] = l;
    }
    const double f2s = Fx * Fx + Fy * Fy + Fz * Fz, s2 = sig.re * sig.re + sig.im * sig.im;
    e = ekin * ie2 + 0.5 * (g0 * n * n + g1 * f2s + g2 * s2 / 5.0) + vmu * n;
    en = 0.5 * n * n;
    ef = 0.5 * f2s;
    es = 0.1 * s2;
    e *= meas; en *= meas; ef *= meas; es *= meas;
  }
  // four partials in a 6-double slot per chunk: two block sums (e, en, ef) and (es, 0, 0)
  block_sum3(e, en, ef, part + 6 * (int64_t)r.c);
  __syncthreads();
  block_sum3(es, 0.0, 0.0, part + 6 * (int64_t)r.c + 3);
}

// Fidelity objective, pass 1: chunk partials of eps^d <target|psi> (re, im).
template <typename T>
__global__ __launch_bounds__(kChunk) void k_fid_overlap(const cx<T>* __restrict__ st, const cx<T>* __restrict__ tgt,
                                                       LaunchGeom g, double meas, double* __restrict__ part) {
  const Site r = site_here(g);
  double re = 0.0, im = 0.0;
  if (r.ok) {
    cx<double> a[5], b[5];
    load_site(st, r.d, r.s, a, b);
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const cx<T> tv = tgt[r.d.psi_off + (int64_t)m * r.d.sites + r.s];
      const cx<double> t{(double)tv.re, (double)tv.im};
      const cx<double> c = cmulc(t, a[m] + b[m]);
      re += c.re;
      im += c.im;
    }
    re *= meas;
    im *= meas;
  }
  block_sum3(re, im, 0.0, part + 3 * (int64_t)r.c);
}

// Per-instance sum of the pass-1 partials into ov[inst][3].
__global__ __launch_bounds__(kChunk) void k_fid_reduce(LaunchGeom g, const double* __restrict__ part,
                                                      double* __restrict__ ov) {
  const InstDesc d = g.inst[blockIdx.x];
  double v[3] = {0.0, 0.0, 0.0};
  for (int c = threadIdx.x; c < d.nchunks; c += kChunk) {
    v[0] += part[3 * (d.chunk_begin + c)];
    v[1] += part[3 * (d.chunk_begin + c) + 1];
  }
  block_sum3(v[0], v[1], v[2], ov + 3 * (int64_t)blockIdx.x);
}

// Pass 2: lambda_a = lambda_b = 2 eps^d <target|psi> target.
template <typename T>
__global__ __launch_bounds__(kChunk) void k_fid_grad(const cx<T>* __restrict__ tgt, cx<double>* __restrict__ lam,
                                                    LaunchGeom g, double meas, const double* __restrict__ ov) {
  const Site r = site_here(g);
  if (!r.ok) return;
  const int inst = g.chunk2inst[r.c];
  const cx<double> o{ov[3 * inst], ov[3 * inst + 1]};
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const cx<T> tv = tgt[r.d.psi_off + (int64_t)m * r.d.sites + r.s];
    const cx<double> l = (2.0 * meas) * (o * cx<double>{(double)tv.re, (double)tv.im});
    const int64_t off = r.d.qb_off + (int64_t)m * r.d.sites + r.s;
    lam[off] = l;
    lam[off + 5 * (int64_t)r.d.sites] = l;
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
#define QLG_GRID dim3(g.nchunks), dim3(kChunk), 0, st

hipError_t launch_chain(int dtype, const void* in, void* out, void* rec, const LaunchGeom& g, int axis, int qb,
                        bool with_u, double tg0, double tg1, double tg25, const ExtPot& ext, double theta,
                        hipStream_t st) {
  if (g.nchunks == 0) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(k_chain<float>, QLG_GRID, (const cx<float>*)in, (cx<float>*)out, (cx<float>*)rec, g, axis,
                       qb, with_u ? 1 : 0, Angles<float>{(float)tg0, (float)tg1, (float)tg25}, ext.V, ext.mu,
                       theta);
  else
    hipLaunchKernelGGL(k_chain<double>, QLG_GRID, (const cx<double>*)in, (cx<double>*)out, (cx<double>*)rec, g,
                       axis, qb, with_u ? 1 : 0, Angles<double>{tg0, tg1, tg25}, ext.V, ext.mu, theta);
  return hipGetLastError();
}

hipError_t launch_sub_iprime_adj(const void* in, void* out, const LaunchGeom& g, int axis, int qb, hipStream_t st) {
  hipLaunchKernelGGL(k_sub_iprime_adj, QLG_GRID, (const cx<double>*)in, (cx<double>*)out, g, axis, qb);
  return hipGetLastError();
}

hipError_t launch_sub_vjp(int dtype, const void* z, void* lam, const LaunchGeom& g, double theta, double g0,
                          double g1, double g2, const ExtPot& ext, double* part, double* acc, hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_sub_vjp<float>, QLG_GRID, (const cx<float>*)z, (cx<double>*)lam, g, theta, g0, g1, g2,
                       ext.V, ext.mu, part);
  else
    hipLaunchKernelGGL(k_sub_vjp<double>, QLG_GRID, (const cx<double>*)z, (cx<double>*)lam, g, theta, g0, g1,
                       g2, ext.V, ext.mu, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dg_accumulate, dim3(1), dim3(kDgThreads), 0, st, (const double*)part, g.nchunks, acc);
  return hipGetLastError();
}

hipError_t launch_sub_adj(int dtype, const void* z, const void* lam_in, void* lam_out, const LaunchGeom& g, int axis,
                          int qb, double theta, double g0, double g1, double g2, const ExtPot& ext, double* part,
                          hipStream_t st) {
  if (g.nchunks == 0) return hipSuccess;
  const dim3 grid(g.nchunks * (kChunk / kLanes)), block(kLanes);
  if (dtype == 0)
    hipLaunchKernelGGL(k_sub_adj<float>, grid, block, 0, st, (const cx<float>*)z, (const cx<double>*)lam_in,
                       (cx<double>*)lam_out, g, axis, qb, theta, g0, g1, g2, ext.V, ext.mu, part);
  else
    hipLaunchKernelGGL(k_sub_adj<double>, grid, block, 0, st, (const cx<double>*)z, (const cx<double>*)lam_in,
                       (cx<double>*)lam_out, g, axis, qb, theta, g0, g1, g2, ext.V, ext.mu, part);
  return hipGetLastError();
}

hipError_t launch_chain_x4(int dtype, const void* in, void* out, void* const rec[4], const LaunchGeom& g,
                           const int* xpre, int nwaves, double tg0, double tg1, double tg25, const ExtPot& ext,
                           double theta, hipStream_t st) {
  if (nwaves <= 0) return hipSuccess;
  constexpr int kWaves = kChunk / kLanes;
  const dim3 grid((nwaves + kWaves - 1) / kWaves), block(kChunk);
  if (dtype == 0)
    hipLaunchKernelGGL(k_chain_x4<float>, grid, block, 0, st, (const cx<float>*)in, (cx<float>*)out,
                       (cx<float>*)rec[0], (cx<float>*)rec[1], (cx<float>*)rec[2], (cx<float>*)rec[3], g, xpre,
                       nwaves, Angles<float>{(float)tg0, (float)tg1, (float)tg25}, ext.V, ext.mu, theta);
  else
    hipLaunchKernelGGL(k_chain_x4<double>, grid, block, 0, st, (const cx<double>*)in, (cx<double>*)out,
                       (cx<double>*)rec[0], (cx<double>*)rec[1], (cx<double>*)rec[2], (cx<double>*)rec[3], g,
                       xpre, nwaves, Angles<double>{tg0, tg1, tg25}, ext.V, ext.mu, theta);
  return hipGetLastError();
}

hipError_t launch_x4_prefix(const LaunchGeom& g, int* xpre, hipStream_t st) {
  hipLaunchKernelGGL(k_x4_prefix, dim3(1), dim3(64), 0, st, g, xpre);
  return hipGetLastError();
}

hipError_t launch_adj_x4(int dtype, const void* const z[4], const void* lam_in, void* lam_out, const LaunchGeom& g,
                         const int* xpre, int nwaves, double theta, double g0, double g1, double g2,
                         const ExtPot& ext, double* part, hipStream_t st) {
  if (nwaves <= 0) return hipSuccess;
  constexpr int kWaves = kChunk / kLanes;
  // one wavefront per SIMD: at most one workgroup of four per CU, each walking several tiles
  constexpr int kAdjX4Blocks = 256;
  const dim3 grid(std::min((nwaves + kWaves - 1) / kWaves, kAdjX4Blocks)), block(kChunk);
  const double* pot = ext.V;
  if (dtype == 0)
    hipLaunchKernelGGL(k_adj_x4<float>, grid, block, 0, st, (const cx<float>*)z[0], (const cx<float>*)z[1],
                       (const cx<float>*)z[2], (const cx<float>*)z[3], (const cx<double>*)lam_in,
                       (cx<double>*)lam_out, g, xpre, nwaves, theta, g0, g1, g2, pot, ext.mu, part);
  else
    hipLaunchKernelGGL(k_adj_x4<double>, grid, block, 0, st, (const cx<double>*)z[0], (const cx<double>*)z[1],
                       (const cx<double>*)z[2], (const cx<double>*)z[3], (const cx<double>*)lam_in,
                       (cx<double>*)lam_out, g, xpre, nwaves, theta, g0, g1, g2, pot, ext.mu, part);
  return hipGetLastError();
}

hipError_t launch_dg_reduce(const double* part, int64_t nparts, double* red, double* acc, hipStream_t st) {
  hipLaunchKernelGGL(k_dg_blocks, dim3(kDgBlocks), dim3(kChunk), 0, st, part, nparts, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_dg_accumulate(red, kDgBlocks, acc, st);
}

hipError_t launch_dg_accumulate(const double* part, int nparts, double* acc, hipStream_t st) {
  hipLaunchKernelGGL(k_dg_accumulate, dim3(1), dim3(kDgThreads), 0, st, part, nparts, acc);
  return hipGetLastError();
}

hipError_t launch_energy_grad(int dtype, int ndim, const void* state, void* lam, const LaunchGeom& g, double eps,
                              double g0, double g1, double g2, const ExtPot& ext, double* part, hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_energy_grad<float>, QLG_GRID, (const cx<float>*)state, (cx<double>*)lam, g, ndim, eps,
                       g0, g1, g2, ext.V, ext.mu, part);
  else
    hipLaunchKernelGGL(k_energy_grad<double>, QLG_GRID, (const cx<double>*)state, (cx<double>*)lam, g, ndim,
                       eps, g0, g1, g2, ext.V, ext.mu, part);
  return hipGetLastError();
}

hipError_t launch_fidelity_grad(int dtype, const void* state, const void* target, void* lam, const LaunchGeom& g,
                                double meas, double* part, double* ov, hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_fid_overlap<float>, QLG_GRID, (const cx<float>*)state, (const cx<float>*)target, g, meas,
                       part);
  else
    hipLaunchKernelGGL(k_fid_overlap<double>, QLG_GRID, (const cx<double>*)state, (const cx<double>*)target, g,
                       meas, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fid_reduce, dim3(g.nbatch), dim3(kChunk), 0, st, g, (const double*)part, ov);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (dtype == 0)
    hipLaunchKernelGGL(k_fid_grad<float>, QLG_GRID, (const cx<float>*)target, (cx<double>*)lam, g, meas,
                       (const double*)ov);
  else
    hipLaunchKernelGGL(k_fid_grad<double>, QLG_GRID, (const cx<double>*)target, (cx<double>*)lam, g, meas,
                       (const double*)ov);
  return hipGetLastError();
}

// complex128 cotangent: canonical qubits layout <-> padded planes
__global__ __launch_bounds__(kChunk) void k_lam_in(const cx<double>* __restrict__ qb, cx<double>* __restrict__ st,
                                                  LaunchGeom g) {
  const Site r = site_here(g);
  if (!r.ok) return;
#pragma unroll
  for (int p = 0; p < 10; ++p) st[r.d.off + p * r.d.stride + r.s] = qb[r.d.qb_off + (int64_t)p * r.d.sites + r.s];
}
__global__ __launch_bounds__(kChunk) void k_lam_out(const cx<double>* __restrict__ st, cx<double>* __restrict__ qb,
                                                   LaunchGeom g) {
  const Site r = site_here(g);
  if (!r.ok) return;
#pragma unroll
  for (int p = 0; p < 10; ++p) qb[r.d.qb_off + (int64_t)p * r.d.sites + r.s] = st[r.d.off + p * r.d.stride + r.s];
}

// Adjoint of the encoding a = b = psi / 2 (Sec. III, two qubits per m_f level): psi enters
// both qubits with weight 1/2, so dL/dpsi_m = (lambda_a,m + lambda_b,m) / 2.  Canonical
// qubits layout in, canonical psi layout out, both complex128.
__global__ __launch_bounds__(kChunk) void k_encode_adj(const cx<double>* __restrict__ qb,
                                                      cx<double>* __restrict__ dpsi, LaunchGeom g) {
  const Site r = site_here(g);
  if (!r.ok) return;
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const cx<double> la = qb[r.d.qb_off + (int64_t)m * r.d.sites + r.s];
    const cx<double> lb = qb[r.d.qb_off + (int64_t)(5 + m) * r.d.sites + r.s];
    dpsi[r.d.psi_off + (int64_t)m * r.d.sites + r.s] = 0.5 * (la + lb);
  }
}

hipError_t launch_encode_adj(const void* lam, void* dpsi, const LaunchGeom& g, hipStream_t st) {
  hipLaunchKernelGGL(k_encode_adj, QLG_GRID, (const cx<double>*)lam, (cx<double>*)dpsi, g);
  return hipGetLastError();
}

hipError_t launch_lam_layout(bool to_planes, const void* src, void* dst, const LaunchGeom& g, hipStream_t st) {
  if (to_planes)
    hipLaunchKernelGGL(k_lam_in, QLG_GRID, (const cx<double>*)src, (cx<double>*)dst, g);
  else
    hipLaunchKernelGGL(k_lam_out, QLG_GRID, (const cx<double>*)src, (cx<double>*)dst, g);
  return hipGetLastError();
}

__global__ void k_zero(double* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

hipError_t launch_zero(double* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace qlg
