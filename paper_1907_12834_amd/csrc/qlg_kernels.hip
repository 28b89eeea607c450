// HIP kernels of the spin-2 QLG step for gfx950 (CDNA4).
//
// Fused step, 1D: one wavefront owns a tile of 64 consecutive sites, one site
// per lane, with 4*S halo sites on each side for S fused steps (each I' has
// dependency radius one site).  All five (a_m, b_m) pairs of a site stay in
// registers for the whole pass; the +-1 site streams are cross-lane moves.
// Interior lanes are written back once per pass.  Two variants spread a
// lattice too small to fill the chip over twice the lanes: a and b of a tile
// on two wavefronts (k_step1d_pair), or a site's a and b on two neighbouring
// lanes of 32-site tiles (k_step1d_lanes).
//
// Fused step, 2D: one wavefront owns 64 columns (56 interior + 4 halo each
// side) and streams down a band of rows.  The y half of the step (Sec. VII
// schedule: U, I'_{y,b}, U, I'_{y,b}, U, I'_{y,a}, U, I'_{y,a}) is a four-stage
// software pipeline along the row loop: each stage keeps one row of pending
// amplitudes in registers, so the y streams never leave the lane.  A row that
// leaves the last stage runs the x half (U, I'_{x,b}, ..., I'_{x,a}) across
// lanes and is stored.  One HBM read and one write per site per step, plus
// the halo rows and columns.
//
// The self-interaction U (qlg_math.hpp) is the arithmetic core: the path is
// bound by the vector ALUs, not by HBM, and uses no matrix cores.

#include <hip/hip_ext.h>

#include <cmath>

#include "qlg_internal.hpp"
#include "qlg_math.hpp"

namespace qlg {

// Whole-wavefront moves by one lane through DPP (wave_shl:1, wave_shr:1, both
// available on CDNA): a VALU operation that the compiler can fold into the
// arithmetic that consumes it, instead of a round trip through the LDS
// crossbar.  The end lane, always a halo lane here, reads 0.
constexpr int kDppWaveShl1 = 0x130;   // lane i reads lane i + 1
constexpr int kDppWaveShr1 = 0x138;   // lane i reads lane i - 1

template <int Ctrl>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), Ctrl, 0xF, 0xF, true));
}
template <int Ctrl>
__device__ __forceinline__ double dpp_move(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, Ctrl, 0xF, 0xF, true);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), Ctrl, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <typename T>
__device__ __forceinline__ cx<T> from_next_lane(cx<T> v) {
  return cx<T>{dpp_move<kDppWaveShl1>(v.re), dpp_move<kDppWaveShl1>(v.im)};
}
template <typename T>
__device__ __forceinline__ cx<T> from_prev_lane(cx<T> v) {
  return cx<T>{dpp_move<kDppWaveShr1>(v.re), dpp_move<kDppWaveShr1>(v.im)};
}

// 4 I'_{x,q} = S_q (2C) S_q^T (2C) with lanes along x (the factor 1/4 is left to
// the caller).  Q = 1: qubit b (the paper's qubit 2) moves; Q = 0: qubit a (qubit 1).
template <typename T, int Q>
__device__ __forceinline__ void iprime4_lanes(cx<T> (&a)[5], cx<T> (&b)[5]) {
  collide2(a, b);
#pragma unroll
  for (int m = 0; m < 5; ++m) {   // S^T: q(x) <- q(x + 1)
    if (Q) b[m] = from_next_lane(b[m]);
    else   a[m] = from_next_lane(a[m]);
  }
  collide2(a, b);
#pragma unroll
  for (int m = 0; m < 5; ++m) {   // S: q(x) <- q(x - 1)
    if (Q) b[m] = from_prev_lane(b[m]);
    else   a[m] = from_prev_lane(a[m]);
  }
}

// Angles of interleaved substep j = 0..3 of a four-I' sequence, on a state that
// carries the factor 4^j of the j I' before it: the n terms' angles and F's scale
// times 16^-j (exact).  Formed from the unscaled angles in registers, so that a
// run-time j reads no kernel argument inside the row loop.
template <typename T>
__device__ __forceinline__ Angles<T> substep_angles(const Angles<T>& base, int j) {
  const T f = ldexp(T(1), -4 * j);
  Angles<T> a = base;
  a.tg0 *= f;
  a.tg25 *= f;
  a.fs = f;
  return a;
}

__device__ __forceinline__ int64_t wrap64(int64_t x, int64_t n) {
  int64_t r = x % n;
  return r < 0 ? r + n : r;
}

// Sum over the 64 lanes of a wavefront (every lane returns the total).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kLanes);
  return v;
}

// Row access of the 2D kernel through buffer resources.  A resource covers one row of one
// amplitude plane (base and record count are wavefront-uniform, in scalar registers); a lane
// passes its byte offset in the row.  The hardware drops a store whose offset is at or beyond
// the record count and returns 0 for such a load, so a lane or a row with nothing to write
// still issues its store, without a branch: every path through the row loop then issues the
// same memory instructions, and the compiler's wait for the row loaded ahead does not also
// wait for the stores of the row before it.
constexpr int kBufWord3 = 0x00020000;   // resource word 3 on gfx9: 32-bit data format, no swizzle
constexpr uint32_t kOffNone = 0x80000000u;

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const cx<T>* row, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<cx<T>*>(row), (short)0, (int)bytes, kBufWord3);
}
__device__ __forceinline__ cx<float> buf_load(const cx<float>*, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(cx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ cx<double> buf_load(const cx<double>*, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(cx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}
__device__ __forceinline__ void buf_store(cx<float> v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
}
__device__ __forceinline__ void buf_store(cx<double> v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, (int)off, 0, 0);
}

// Kernel arguments shared by the fused step kernels.
template <typename T>
struct StepArgs {
  const cx<T>* __restrict__ in;
  cx<T>* __restrict__ out;
  const InstDesc* __restrict__ inst;
  const int32_t* __restrict__ tile2inst;
  double* __restrict__ ovpart;   // [ntiles][2] overlap partials (written when overlap != 0)
  Angles<T> ang;                 // interleaved U^{1/(4d)}, theta = eps^2 / (4 d), unscaled state
                                 // (substep_angles scales it for substep j of a four-I' sequence)
  Angles<T> ang_full;            // plain split: theta = eps^2, unscaled state
  const double* __restrict__ pot;  // V(x), canonical scalar layout (nullptr: none); kExt kernels only
  double mu;                     // chemical potential; kExt kernels only
  T th_ext;                      // theta of the (V + mu) phase: eps^2/(4d), or eps^2 for the plain split
  const cx<T>* prev;             // 2D/3D: the state before the step (overlap); may equal out
  int32_t zpass;                 // 3D: this launch is the z pass (four z substeps only)
  int32_t plain_u;               // plain split: this launch applies the step's single U
  int32_t ntiles;
  int32_t steps;                 // 1D: steps fused in this pass
  int32_t tile_rows;             // 2D: rows per streaming tile
  int32_t plain;                 // 1: plain split, 0: interleaved
  int32_t overlap;               // 1: record <psi_t|psi_{t-1}> of the last step
};

// theta (V + mu) at site s of instance d: the per-site angle of the (V + mu) phase
template <typename T>
__device__ __forceinline__ T ext_angle(const StepArgs<T>& A, const InstDesc& d, int64_t s) {
  return A.th_ext * T((A.pot ? A.pot[d.psi_off / 5 + s] : 0.0) + A.mu);
}

// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each with its
// own L2.  Give each XCD a contiguous range of logical workgroups, so that tiles
// that share halo rows and columns (consecutive tiles) read them through one L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_contiguous_block(int b, int nblocks) {
  const int x = b % kXcds, l = b / kXcds;
  const int per = nblocks / kXcds, extra = nblocks % kXcds;
  return x * per + (x < extra ? x : extra) + l;
}

// ---------------------------------------------------------------------------
// 1D fused step: `steps` steps per pass, 4*steps halo sites on each side
// ---------------------------------------------------------------------------
// Substep k = 0..3 of a 1D step is [U] I'_{x,q} with q = b, b, a, a (Sec. VII:
// psi(t+tau) = I'_1 U I'_1 U I'_2 U I'_2 U psi(t), rightmost first); the plain
// split applies one U with theta = eps^2 before the first I' only.
template <typename T, bool kExt>
__global__ __launch_bounds__(256) void k_step1d(StepArgs<T> A) {
  const int w = xcd_contiguous_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (w >= A.ntiles) return;   // whole wavefronts only; no block-level synchronisation below
  const int lane = threadIdx.x & (kLanes - 1);
  const InstDesc d = A.inst[A.tile2inst[w]];
  const int H = 4 * A.steps;
  const int TV = kLanes - 2 * H;
  const int64_t L = d.nx;
  const int64_t x = (int64_t)(w - d.tile_begin) * TV - H + lane;
  const int64_t xw = wrap64(x, L);
  const cx<T>* src = A.in + d.off + xw;
  cx<T> a[5], b[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    a[m] = src[m * d.stride];
    b[m] = src[(5 + m) * d.stride];
  }
  // each lane keeps its site for the whole pass: one (V + mu) angle per lane
  T ext = T(0);
  if constexpr (kExt) ext = ext_angle(A, d, xw);
  const bool plain = A.plain != 0;
  cx<T> pold[5];
  // one step: [U] I'_{x,b} [U] I'_{x,b} [U] I'_{x,a} [U] I'_{x,a}; the moving qubit is
  // a compile-time parameter of each inner loop.  The four I' factors 1/4 are
  // applied together at the end of the step (exact); U in between sees the state
  // scaled by 4^j and compensates through its angles.
#pragma unroll 1
  for (int st = 0; st < A.steps; ++st) {
    if (A.overlap && st == A.steps - 1) {
#pragma unroll
      for (int m = 0; m < 5; ++m) pold[m] = a[m] + b[m];
    }
#pragma unroll 1
    for (int j = 0; j < 2; ++j) {
      if (!plain || j == 0) potential<T, kExt>(a, b, plain ? A.ang_full : substep_angles(A.ang, j), ext);
      iprime4_lanes<T, 1>(a, b);
    }
#pragma unroll 1
    for (int j = 2; j < 4; ++j) {
      if (!plain) potential<T, kExt>(a, b, substep_angles(A.ang, j), ext);
      iprime4_lanes<T, 0>(a, b);
    }
    scale_by(a, b, T(1.0 / 256.0));
  }
  const bool valid = lane >= H && lane < kLanes - H && x < L;
  if (valid) {
    cx<T>* dst = A.out + d.off + x;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      dst[m * d.stride] = a[m];
      dst[(5 + m) * d.stride] = b[m];
    }
  }
  if (A.overlap) {
    double ore = 0.0, oim = 0.0;
    if (valid) {
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const cx<T> c = cmulc(a[m] + b[m], pold[m]);   // conj(psi_t) psi_{t-1}
        ore += (double)c.re;
        oim += (double)c.im;
      }
    }
    ore = wave_sum(ore);
    oim = wave_sum(oim);
    if (lane == 0) {
      A.ovpart[2 * w] = ore;
      A.ovpart[2 * w + 1] = oim;
    }
  }
}

// ---------------------------------------------------------------------------
// 1D fused step, qubit pair on two wavefronts
// ---------------------------------------------------------------------------
// Same tiles and schedule as k_step1d, but a tile's a (the paper's qubit 1) and
// b (qubit 2) live on two wavefronts (even and odd wave of the workgroup; two
// tiles per workgroup of four waves), so a lattice too small to fill the chip
// runs on twice as many SIMDs with about 0.7x the per-lane work.  The partner
// amplitudes come through LDS.
//
// Each substep U I'_{x,Q} is evaluated as C U S^T C then S: the collide
// commutes with U (it mixes a and b with scalar weights, and W acts on the m
// index of both alike) and leaves psi = a + b unchanged, so the first collide
// and the coefficients of W share one exchange, and the second collide takes
// the other.  In exact arithmetic the result is the step of k_step1d.
//
// own' of the unnormalised collide, on either wave: with s = own + other and
// e = own - other, own' = (s_re + e_im, s_im - e_re).  For own = a this is 2a',
// for own = b (e = -(a - b) exactly) it is 2b'.
template <typename T>
__device__ __forceinline__ void collide_own(cx<T> (&x)[5], const cx<T> (&y)[5]) {
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const T sr = x[m].re + y[m].re, si = x[m].im + y[m].im;
    const T er = x[m].re - y[m].re, ei = x[m].im - y[m].im;
    x[m] = cx<T>{sr + ei, si - er};
  }
}

constexpr int kPairTiles = 2;                 // tiles per pair workgroup
constexpr int kPairWaves = 2 * kPairTiles;    // wavefronts per pair workgroup

// LDS exchange between the two wavefronts of a tile: double-buffered, one
// workgroup barrier per exchange (the buffer written now was last read before
// the previous barrier).  Wave v of the workgroup owns slot v; its partner is v ^ 1.
template <typename T>
struct PairXchg {
  T (*buf)[kPairWaves][10][kLanes];
  int q, v, lane, cur;
  __device__ __forceinline__ void swap(const cx<T> (&own)[5], cx<T> (&other)[5]) {
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      buf[cur][v][2 * m][lane] = own[m].re;
      buf[cur][v][2 * m + 1][lane] = own[m].im;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 5; ++m) other[m] = cx<T>{buf[cur][v ^ 1][2 * m][lane], buf[cur][v ^ 1][2 * m + 1][lane]};
    cur ^= 1;
  }
  // S^T (Up: q(x) <- q(x + 1)) or S (q(x) <- q(x - 1)) when this wave holds the
  // streaming qubit Q (uniform per wavefront): one lane per site
  template <int Q, bool Up>
  __device__ __forceinline__ void stream(cx<T> (&x)[5]) const {
    if (q == Q) {
#pragma unroll
      for (int m = 0; m < 5; ++m) x[m] = Up ? from_next_lane(x[m]) : from_prev_lane(x[m]);
    }
  }
};

// One substep [U] I'_{x,Q} on this lane's qubit x (Q: qubit that streams).
template <typename T, int Q, bool kExt, typename Xchg>
__device__ __forceinline__ void pair_substep(cx<T> (&x)[5], Xchg& X, bool with_u, const Angles<T>& ang, T ext) {
  cx<T> y[5];
  X.swap(x, y);
  if (with_u) {
    WCoef<T> W;
    w_coefficients<T, kExt>(x, y, ang, W, ext);   // psi = x + y, the same sum on both holders
    collide_own(x, y);
    w_apply(x, W);
  } else {
    collide_own(x, y);
  }
  X.template stream<Q, true>(x);    // S^T
  X.swap(x, y);
  collide_own(x, y);
  X.template stream<Q, false>(x);   // S
}

template <typename T, bool kExt>
__global__ __launch_bounds__(kLanes * kPairWaves) void k_step1d_pair(StepArgs<T> A) {
  __shared__ T xbuf[2][kPairWaves][10][kLanes];
  // Every wave of the workgroup takes part in every barrier: a workgroup whose
  // second tile lies past the end recomputes the last tile and stores nothing.
  const int v = threadIdx.x >> 6;
  const int q = v & 1;
  const int lane = threadIdx.x & (kLanes - 1);
  const int wt = xcd_contiguous_block(blockIdx.x, gridDim.x) * kPairTiles + (v >> 1);
  const bool real = wt < A.ntiles;
  const int w = real ? wt : A.ntiles - 1;
  const InstDesc d = A.inst[A.tile2inst[w]];
  const int H = 4 * A.steps;
  const int TV = kLanes - 2 * H;
  const int64_t L = d.nx;
  const int64_t x0 = (int64_t)(w - d.tile_begin) * TV - H + lane;
  const int64_t xw = wrap64(x0, L);
  const cx<T>* src = A.in + d.off + (int64_t)(5 * q) * d.stride + xw;
  cx<T> x[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) x[m] = src[m * d.stride];
  PairXchg<T> X{xbuf, q, v, lane, 0};
  T ext = T(0);
  if constexpr (kExt) ext = ext_angle(A, d, xw);
  const bool plain = A.plain != 0;
  cx<T> pold[5];
#pragma unroll 1
  for (int st = 0; st < A.steps; ++st) {
    if (A.overlap && st == A.steps - 1) {
      cx<T> y[5];
      X.swap(x, y);
#pragma unroll
      for (int m = 0; m < 5; ++m) pold[m] = x[m] + y[m];
    }
#pragma unroll 1
    for (int j = 0; j < 2; ++j)
      pair_substep<T, 1, kExt>(x, X, !plain || j == 0, plain ? A.ang_full : substep_angles(A.ang, j), ext);
#pragma unroll 1
    for (int j = 2; j < 4; ++j) pair_substep<T, 0, kExt>(x, X, !plain, substep_angles(A.ang, j), ext);
#pragma unroll
    for (int m = 0; m < 5; ++m) x[m] = T(1.0 / 256.0) * x[m];
  }
  const bool valid = real && lane >= H && lane < kLanes - H && x0 < L;
  if (valid) {
    cx<T>* dst = A.out + d.off + (int64_t)(5 * q) * d.stride + x0;
#pragma unroll
    for (int m = 0; m < 5; ++m) dst[m * d.stride] = x[m];
  }
  if (A.overlap) {
    cx<T> y[5];
    X.swap(x, y);
    if (q == 0 && real) {
      double ore = 0.0, oim = 0.0;
      if (valid) {
#pragma unroll
        for (int m = 0; m < 5; ++m) {
          const cx<T> c = cmulc(x[m] + y[m], pold[m]);   // conj(psi_t) psi_{t-1}
          ore += (double)c.re;
          oim += (double)c.im;
        }
      }
      ore = wave_sum(ore);
      oim = wave_sum(oim);
      if (lane == 0) {
        A.ovpart[2 * w] = ore;
        A.ovpart[2 * w + 1] = oim;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 1D fused step, qubit pair on two lanes
// ---------------------------------------------------------------------------
// A wavefront holds a 32-site tile (4*S halo sites on each side, S <= 3), site i
// of the tile on lanes 2i and 2i+1, one qubit amplitude per lane.  During the two
// substeps that stream qubit Q the even lane holds Q and the odd lane the other
// qubit: the lanes trade qubits before the b substeps and before the a substeps
// (free: the first exchange of a substep fetches the partner anyway, and the
// trade only renames registers).
//
// A substep [U] I'_{x,Q} is evaluated as C U S^T C then S (as in k_step1d_pair),
// and the streams are relabellings as well: after S^T the streaming amplitude
// of site i is the one on lane 2i+2, so the second collide pairs lanes 2i+1 and
// 2i+2 (even lanes read the lane before, odd lanes the lane after), and S puts
// the labels back.  No amplitude moves for a stream; the two exchanges of a
// substep are whole-wavefront DPP moves.  On a lattice too small to fill the
// chip this spends two lanes per site for about 0.7x the instructions per lane,
// without the LDS round trips of the two-wavefront form.
constexpr int kDppQuadSwap = 0xB1;      // quad_perm [1, 0, 3, 2]: lane i reads lane i ^ 1
constexpr int kLaneTile = kLanes / 2;   // sites per wavefront of k_step1d_lanes

template <typename T>
__device__ __forceinline__ cx<T> from_pair_lane(cx<T> v) {
  return cx<T>{dpp_move<kDppQuadSwap>(v.re), dpp_move<kDppQuadSwap>(v.im)};
}

// One substep [U] I'_{x,Q}, the streaming qubit on the even lanes.  Trade: the
// lanes trade qubits first (x becomes the partner's amplitude).
template <typename T, bool kExt, bool Trade>
__device__ __forceinline__ void lanes_substep(cx<T> (&x)[5], bool even, bool with_u, const Angles<T>& ang,
                                              T ext) {
  cx<T> y[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const cx<T> p = from_pair_lane(x[m]);
    if (Trade) {
      y[m] = x[m];
      x[m] = p;
    } else {
      y[m] = p;
    }
  }
  if (with_u) {
    WCoef<T> W;
    w_coefficients<T, kExt>(x, y, ang, W, ext);   // psi = x + y, the same sum on both lanes
    collide_own(x, y);
    w_apply(x, W);
  } else {
    collide_own(x, y);
  }
  // S^T relabels the streaming amplitudes one site down: the partners are now
  // (2i+1, 2i+2).  Every lane makes both moves before the per-lane select: a DPP
  // move inside a branch taken by half the lanes would read switched-off lanes.
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const cx<T> prev = from_prev_lane(x[m]), next = from_next_lane(x[m]);
    y[m] = even ? prev : next;
  }
  collide_own(x, y);
  // S: the labels return to (2i, 2i+1)
}

template <typename T, bool kExt>
__global__ __launch_bounds__(256) void k_step1d_lanes(StepArgs<T> A) {
  const int w = xcd_contiguous_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (w >= A.ntiles) return;   // whole wavefronts only; no block-level synchronisation below
  const int lane = threadIdx.x & (kLanes - 1);
  const bool even = (lane & 1) == 0;
  const int i = lane >> 1;
  const InstDesc d = A.inst[A.tile2inst[w]];
  const int H = 4 * A.steps;
  const int TV = kLaneTile - 2 * H;
  const int64_t L = d.nx;
  const int64_t x0 = (int64_t)(w - d.tile_begin) * TV - H + i;
  const int64_t xw = wrap64(x0, L);
  // between steps a is on the even lanes (the b substeps of a step trade first)
  const int64_t q = even ? 0 : 5;
  const cx<T>* src = A.in + d.off + q * d.stride + xw;
  cx<T> x[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) x[m] = src[m * d.stride];
  T ext = T(0);
  if constexpr (kExt) ext = ext_angle(A, d, xw);
  const bool plain = A.plain != 0;
  cx<T> pold[5];
#pragma unroll 1
  for (int st = 0; st < A.steps; ++st) {
    if (A.overlap && st == A.steps - 1) {
#pragma unroll
      for (int m = 0; m < 5; ++m) pold[m] = x[m] + from_pair_lane(x[m]);
    }
    // substeps j = 2h, 2h + 1 stream b (h = 0), then a (h = 1); the arithmetic is the
    // same for both, the streaming qubit being on the even lanes
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
      lanes_substep<T, kExt, true>(x, even, !plain || h == 0,
                                   plain ? A.ang_full : substep_angles(A.ang, 2 * h), ext);
      lanes_substep<T, kExt, false>(x, even, !plain, substep_angles(A.ang, 2 * h + 1), ext);
    }
#pragma unroll
    for (int m = 0; m < 5; ++m) x[m] = T(1.0 / 256.0) * x[m];
  }
  const bool valid = i >= H && i < kLaneTile - H && x0 < L;
  if (valid) {
    cx<T>* dst = A.out + d.off + q * d.stride + x0;
#pragma unroll
    for (int m = 0; m < 5; ++m) dst[m * d.stride] = x[m];
  }
  if (A.overlap) {
    double ore = 0.0, oim = 0.0;
    cx<T> y[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) y[m] = from_pair_lane(x[m]);
    if (valid && even) {
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const cx<T> c = cmulc(x[m] + y[m], pold[m]);   // conj(psi_t) psi_{t-1}
        ore += (double)c.re;
        oim += (double)c.im;
      }
    }
    ore = wave_sum(ore);
    oim = wave_sum(oim);
    if (lane == 0) {
      A.ovpart[2 * w] = ore;
      A.ovpart[2 * w + 1] = oim;
    }
  }
}

// ---------------------------------------------------------------------------
// 2D fused step: y half as a 4-stage register pipeline along rows, x half across lanes
// ---------------------------------------------------------------------------
// Stage k of the y half is [U] I'_{y,q}, q = b, b, a, a.  The streaming row
// enters stage k as row r of the stage input and leaves as row r - 1 of its
// output.  Each stage keeps two pending 5-vectors per lane:
//   cn: the non-moving qubit of C(input) at row r - 1,
//   mq: the moving qubit after the second collide at row r - 2.
template <typename T, int Q>
__device__ __forceinline__ void y_stage_core(cx<T> (&a)[5], cx<T> (&b)[5], cx<T> (&cn)[5], cx<T> (&mq)[5]) {
  collide2(a, b);                     // c(r)
  cx<T> ta[5], tb[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {       // t(r-1) = (c(r-1).nonq, c(r).q)   [S^T: q(y) <- q(y+1)]
    if (Q) { ta[m] = cn[m]; tb[m] = b[m]; cn[m] = a[m]; }
    else   { ta[m] = a[m]; tb[m] = cn[m]; cn[m] = b[m]; }
  }
  collide2(ta, tb);                   // m(r-1), times 4
#pragma unroll
  for (int m = 0; m < 5; ++m) {       // out(r-1) = (m(r-1).nonq, m(r-2).q)  [S: q(y) <- q(y-1)]
    if (Q) { a[m] = ta[m]; b[m] = mq[m]; mq[m] = tb[m]; }
    else   { a[m] = mq[m]; b[m] = tb[m]; mq[m] = ta[m]; }
  }
}

// One y stage on the streaming row, its pending rows kept in this lane's LDS slot.
template <typename T, int Q>
__device__ __forceinline__ void y_stage_lds(cx<T> (&a)[5], cx<T> (&b)[5], cx<T>* slot) {
  cx<T> cn[5], mq[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    cn[m] = slot[m * kLanes];
    mq[m] = slot[(5 + m) * kLanes];
  }
  y_stage_core<T, Q>(a, b, cn, mq);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    slot[m * kLanes] = cn[m];
    slot[(5 + m) * kLanes] = mq[m];
  }
}

// LDS words per wavefront and y stage of the pipeline: (cn[5], mq[5]) x 64 lanes.
constexpr int kSlotsPerStage = 10;

// Parts of a step (StepPart): a launch of kYFirst or kYSecond keeps a two-stage pipeline,
// half the LDS of the four-stage one, which lets two wavefronts share a SIMD in complex128.
// The state between the two launches is the true state (scale 1).
template <int kPart>
constexpr int stages_of() { return kPart == kWhole ? 4 : 2; }
// Wavefronts per workgroup.  A workgroup of four lands one wavefront on each SIMD of a CU, so
// the SIMDs hold equal numbers of wavefronts; with workgroups of two, the wavefronts of two
// workgroups can share two SIMDs of a CU and leave the other two idle whenever the registers
// allow two per SIMD (the single launch in complex128 2D: 1.63 against 0.95 ms per step; the
// split and the complex64 kernels 1.5-3 % slower).
constexpr int k2DWaves = 4;

// With the y half split, a launch's pipeline leaves LDS for two wavefronts per SIMD: the
// register budget is set to match (256 per lane).
template <typename T, bool kExt, int kPart>
__global__ __launch_bounds__(64 * k2DWaves) __attribute__((amdgpu_waves_per_eu(kPart == kWhole ? 1 : 2)))
void k_step2d(StepArgs<T> A) {
  constexpr int kStages = stages_of<kPart>();
  constexpr int kLag = 2 * kStages;          // rows between a row's load and its store
  // Per-lane pipeline buffers live in LDS; every lane reads back only the
  // slots it wrote itself, so no barrier is needed anywhere in the kernel.
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // the tile and everything derived from it are wavefront-uniform (scalar registers)
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int w = xcd_contiguous_block(blockIdx.x, gridDim.x) * k2DWaves + wv;
  if (w >= A.ntiles) return;
  const int lane = threadIdx.x & (kLanes - 1);
  cx<T>* const my = reinterpret_cast<cx<T>*>(smem_raw) + wv * (kStages * kSlotsPerStage * kLanes) + lane;
  const InstDesc d = A.inst[A.tile2inst[w]];
  // Tile -> (x tile, band, plane).  The rows of a band stream along y (2D, and the y-x
  // pass of a 3D step: one z plane per band) or along z (the z pass of a 3D step: one y
  // plane per band, 64-column tiles without x halo since no x substep follows).
  const bool zp = A.zpass != 0;
  const int t = w - (zp ? d.tile_begin_z : d.tile_begin);
  const int ntx = zp ? d.ntx_z : d.ntx, nband = zp ? d.ntz : d.nty;
  const int tx = t % ntx, tb = t / ntx;
  const int ty = tb % nband, plane = tb / nband;
  const int nx = d.nx;
  const int nrow = zp ? d.nz : d.ny;                                     // extent along the rows
  const int64_t rstride = zp ? (int64_t)d.nx * d.ny : (int64_t)d.nx;     // sites between rows
  const int64_t pbase = zp ? (int64_t)plane * d.nx : (int64_t)plane * d.nx * d.ny;
  const int halo = zp ? 0 : kHalo2D;
  const int x = tx * (kLanes - 2 * halo) - halo + lane;
  const int xw = (int)wrap64(x, nx);
  const int y0 = ty * A.tile_rows;
  const bool xvalid = lane >= halo && lane < kLanes - halo && x < nx;
  const bool plain = A.plain != 0;
  const bool plain_u = A.plain_u != 0;
  // byte offsets of this lane's site in a row: the load's (periodic column) and the
  // store's (beyond any record count for a halo lane or a column past the lattice)
  const uint32_t row_bytes = (uint32_t)nx * (uint32_t)sizeof(cx<T>);
  const uint32_t off_ld = (uint32_t)xw * (uint32_t)sizeof(cx<T>);
  const uint32_t off_st = xvalid ? (uint32_t)x * (uint32_t)sizeof(cx<T>) : kOffNone;
#pragma unroll
  for (int j = 0; j < kStages * kSlotsPerStage; ++j) my[j * kLanes] = cx<T>{T(0), T(0)};

  double ore = 0.0, oim = 0.0;
  const int nrows = A.tile_rows + kLag;
  // Rows are loaded one iteration ahead, so that a row's HBM latency overlaps the
  // arithmetic of the row before it.
  // lattice row of the next load (row y0 - kStages + r of the band, periodic), advanced by
  // one per load instead of a division per row
  int yl = (int)wrap64(y0 - kStages, nrow);
  // with kExt, e is the (V + mu) angle of the row's site in this lane; a load with
  // live == false (after the band's last row) reads nothing and returns zeros
  auto load_row = [&](cx<T>(&a)[5], cx<T>(&b)[5], T& e, bool live) {
    const int64_t s = d.off + pbase + (int64_t)yl * rstride;
    const uint32_t nrec = live ? row_bytes : 0u;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      a[m] = buf_load(A.in, row_rsrc(A.in + s + m * d.stride, nrec), off_ld);
      b[m] = buf_load(A.in, row_rsrc(A.in + s + (5 + m) * d.stride, nrec), off_ld);
    }
    if constexpr (kExt) e = ext_angle(A, d, s - d.off + xw);
    yl = yl + 1 == nrow ? 0 : yl + 1;
  };
  // Stores of lattice row yo; a row outside the lattice (or a row still in the pipeline,
  // live == false) has record count 0, so its stores write nothing.
  auto store_row = [&](const cx<T>(&a)[5], const cx<T>(&b)[5], int yo, bool live) {
    const bool on = live && yo >= 0 && yo < nrow;
    const int64_t s = d.off + pbase + (int64_t)(on ? yo : 0) * rstride;
    const uint32_t nrec = on ? row_bytes : 0u;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      buf_store(a[m], row_rsrc(A.out + s + m * d.stride, nrec), off_st);
      buf_store(b[m], row_rsrc(A.out + s + (5 + m) * d.stride, nrec), off_st);
    }
  };
  // (V + mu) angles: stage i of this launch works on the row loaded i iterations ago,
  // the x half on the row loaded kStages iterations ago
  T er[kStages + 1];
#pragma unroll
  for (int i = 0; i <= kStages; ++i) er[i] = T(0);
  T ne = T(0);
  cx<T> na[5], nb[5];
  load_row(na, nb, ne, true);
  {
    // the stores of a row that writes nothing, so that the loop is entered, as it is
    // re-entered, with one row of stores issued after the row loaded ahead
    const cx<T> z[5] = {};
    store_row(z, z, 0, false);
  }
#pragma unroll 1
  for (int r = 0; r < nrows; ++r) {
    cx<T> a[5], b[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      a[m] = na[m];
      b[m] = nb[m];
    }
    const T en = ne;
    __builtin_amdgcn_sched_barrier(0);
    load_row(na, nb, ne, r + 1 < nrows);
    if constexpr (kExt) {
#pragma unroll
      for (int i = kStages; i > 0; --i) er[i] = er[i - 1];
      er[0] = en;
    }
    // y half: stages (y,b), (y,b), (y,a), (y,a), each [U] I'_y, all four or two of them in
    // this launch; slot i of this lane's LDS holds stage i's pending rows.  The plain split
    // applies its single U at the step's first stage.  Stage i leaves its output times 4
    // (the factor 1/4 of its I' is deferred): all rows pass the same stages, so pending and
    // streaming rows carry the same scale, and the U of stage i takes angles for a state
    // times 4^i; one exact multiplication ends each half.
    if constexpr (kPart != kYSecond) {
#pragma unroll 1
      for (int i = 0; i < 2; ++i) {
        if (!plain || (i == 0 && plain_u))
          potential<T, kExt>(a, b, plain ? A.ang_full : substep_angles(A.ang, i), i == 0 ? er[0] : er[1]);
        y_stage_lds<T, 1>(a, b, my + i * kSlotsPerStage * kLanes);
      }
    }
    if constexpr (kPart != kYFirst) {
      constexpr int i0 = kPart == kWhole ? 2 : 0;
#pragma unroll 1
      for (int i = i0; i < i0 + 2; ++i) {
        if (!plain) potential<T, kExt>(a, b, substep_angles(A.ang, i), i == i0 ? er[i0] : er[i0 + 1]);
        y_stage_lds<T, 0>(a, b, my + i * kSlotsPerStage * kLanes);
      }
    }
    // The row leaving the pipeline is complete from r = kLag on.  The pipeline fill issues
    // the same stores, all dropped, so that every path through the loop issues the same
    // memory instructions in the same order.
    const int yo = y0 - kLag + r;
    const bool done = r >= kLag;
    if (done) {
      scale_by(a, b, T(kStages == 4 ? 1.0 / 256.0 : 1.0 / 16.0));
      if (kPart != kYFirst && !zp) {     // x half (not after the b stages, not in a z pass)
#pragma unroll 1
        for (int j = 0; j < 2; ++j) {
          if (!plain) potential<T, kExt>(a, b, substep_angles(A.ang, j), er[kStages]);
          iprime4_lanes<T, 1>(a, b);
        }
#pragma unroll 1
        for (int j = 2; j < 4; ++j) {
          if (!plain) potential<T, kExt>(a, b, substep_angles(A.ang, j), er[kStages]);
          iprime4_lanes<T, 0>(a, b);
        }
        scale_by(a, b, T(1.0 / 256.0));
        if (A.overlap && yo < nrow) {
          // the state before the step at this site; in a step of several launches it is the
          // location this lane writes below (and no other lane reads or writes it), so it is
          // read first.  Halo lanes read zeros and add nothing.
          const int64_t s = d.off + pbase + (int64_t)yo * rstride;
#pragma unroll
          for (int m = 0; m < 5; ++m) {
            const cx<T> po = buf_load(A.prev, row_rsrc(A.prev + s + m * d.stride, row_bytes), off_st) +
                             buf_load(A.prev, row_rsrc(A.prev + s + (5 + m) * d.stride, row_bytes), off_st);
            const cx<T> c = cmulc(a[m] + b[m], po);
            if (xvalid) {
              ore += (double)c.re;
              oim += (double)c.im;
            }
          }
        }
      }
    }
    store_row(a, b, yo, done);
  }
  if (A.overlap) {
    ore = wave_sum(ore);
    oim = wave_sum(oim);
    if (lane == 0) {
      A.ovpart[2 * w] = ore;
      A.ovpart[2 * w + 1] = oim;
    }
  }
}

// ---------------------------------------------------------------------------
// Elementwise layout kernels (one thread per site, 256-site chunks per instance)
// ---------------------------------------------------------------------------
struct SiteRef {
  InstDesc d;
  int s;
  bool ok;
};

__device__ __forceinline__ SiteRef site_of(const LaunchGeom& g) {
  SiteRef r;
  const int c = blockIdx.x;
  r.d = g.inst[g.chunk2inst[c]];
  r.s = (c - r.d.chunk_begin) * kChunk + threadIdx.x;
  r.ok = r.s < r.d.sites;
  return r;
}

template <typename T>
__global__ __launch_bounds__(kChunk) void k_set_psi(const cx<T>* __restrict__ psi, cx<T>* __restrict__ st,
                                                   LaunchGeom g) {
  const SiteRef r = site_of(g);
  if (!r.ok) return;
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const cx<T> v = T(0.5) * psi[r.d.psi_off + (int64_t)m * r.d.sites + r.s];
    st[r.d.off + m * r.d.stride + r.s] = v;
    st[r.d.off + (5 + m) * r.d.stride + r.s] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(kChunk) void k_get_psi(const cx<T>* __restrict__ st, cx<T>* __restrict__ psi,
                                                   LaunchGeom g) {
  const SiteRef r = site_of(g);
  if (!r.ok) return;
#pragma unroll
  for (int m = 0; m < 5; ++m)
    psi[r.d.psi_off + (int64_t)m * r.d.sites + r.s] =
        st[r.d.off + m * r.d.stride + r.s] + st[r.d.off + (5 + m) * r.d.stride + r.s];
}

template <typename T>
__global__ __launch_bounds__(kChunk) void k_set_qubits(const cx<T>* __restrict__ qb, cx<T>* __restrict__ st,
                                                      LaunchGeom g) {
  const SiteRef r = site_of(g);
  if (!r.ok) return;
#pragma unroll
  for (int p = 0; p < 10; ++p)
    st[r.d.off + p * r.d.stride + r.s] = qb[r.d.qb_off + (int64_t)p * r.d.sites + r.s];
}

template <typename T>
__global__ __launch_bounds__(kChunk) void k_get_qubits(const cx<T>* __restrict__ st, cx<T>* __restrict__ qb,
                                                      LaunchGeom g) {
  const SiteRef r = site_of(g);
  if (!r.ok) return;
#pragma unroll
  for (int p = 0; p < 10; ++p)
    qb[r.d.qb_off + (int64_t)p * r.d.sites + r.s] = st[r.d.off + p * r.d.stride + r.s];
}

// ---------------------------------------------------------------------------
// Observables: per-chunk partial sums (FP64), then per-instance sums
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_sum_store(double (&v)[kNObs], double* __restrict__ dst) {
  __shared__ double red[kNObs][kChunk / kLanes];
  const int lane = threadIdx.x & (kLanes - 1), wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kNObs; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) red[k][wv] = s;
  }
  __syncthreads();
  if (threadIdx.x < kNObs) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kChunk / kLanes; ++j) s += red[threadIdx.x][j];
    dst[threadIdx.x] = s;
  }
}

template <typename T>
__device__ __forceinline__ void load_psi_d(const cx<T>* __restrict__ st, const InstDesc& d, int s,
                                           double (&pr)[5], double (&pi)[5], double* nq) {
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const cx<T> a = st[d.off + m * d.stride + s];
    const cx<T> b = st[d.off + (5 + m) * d.stride + s];
    acc += (double)a.re * a.re + (double)a.im * a.im + (double)b.re * b.re + (double)b.im * b.im;
    pr[m] = (double)a.re + (double)b.re;
    pi[m] = (double)a.im + (double)b.im;
  }
  if (nq) *nq = acc;
}

template <typename T>
__global__ __launch_bounds__(kChunk) void k_observables(const cx<T>* __restrict__ st, LaunchGeom g, int ndim,
                                                       double g0, double g1, double g2,
                                                       const double* __restrict__ pot, double mu,
                                                       double* __restrict__ part) {
  const SiteRef r = site_of(g);
  double v[kNObs];
#pragma unroll
  for (int k = 0; k < kNObs; ++k) v[k] = 0.0;
  if (r.ok) {
    const InstDesc& d = r.d;
    double pr[5], pi[5], nq;
    load_psi_d(st, d, r.s, pr, pi, &nq);
    const int plane = d.nx * d.ny;
    const int x = r.s % d.nx, y = (r.s / d.nx) % d.ny, z = r.s / plane;
    double q[5], n = 0.0;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      q[m] = pr[m] * pr[m] + pi[m] * pi[m];
      n += q[m];
    }
    v[0] = nq;
    v[1] = n;
#pragma unroll
    for (int m = 0; m < 5; ++m) v[2 + m] = q[m];
    // kinetic: forward differences along x (and y, z), periodic
    double ek = 0.0;
    auto add_diff = [&](int sn) {
      double nr[5], ni[5];
      load_psi_d<T>(st, d, sn, nr, ni, nullptr);
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const double dr = nr[m] - pr[m], di = ni[m] - pi[m];
        ek += dr * dr + di * di;
      }
    };
    add_diff(r.s - x + (x + 1 == d.nx ? 0 : x + 1));
    if (ndim >= 2) add_diff(r.s + ((y + 1 == d.ny ? 0 : y + 1) - y) * d.nx);
    if (ndim == 3) add_diff(r.s + ((z + 1 == d.nz ? 0 : z + 1) - z) * plane);
    v[7] = ek;
    // interaction energy density (g0 n^2 + g1 |F|^2 + g2 |sigma|^2 / 5) / 2
    const double r6 = Consts::r6;
    const double Fz = 2.0 * (q[0] - q[4]) + (q[1] - q[3]);
    // F_x + i F_y = 2 p2* p1 + sqrt6 p1* p0 + sqrt6 p0* p-1 + 2 p-1* p-2
    auto cre = [&](int i, int j) { return pr[i] * pr[j] + pi[i] * pi[j]; };
    auto cim = [&](int i, int j) { return pr[i] * pi[j] - pi[i] * pr[j]; };
    const double Fx = 2.0 * (cre(0, 1) + cre(3, 4)) + r6 * (cre(1, 2) + cre(2, 3));
    const double Fy = 2.0 * (cim(0, 1) + cim(3, 4)) + r6 * (cim(1, 2) + cim(2, 3));
    // sigma = 2 p2 p-2 - 2 p1 p-1 + p0^2
    const double sr = 2.0 * (pr[0] * pr[4] - pi[0] * pi[4]) - 2.0 * (pr[1] * pr[3] - pi[1] * pi[3]) +
                      (pr[2] * pr[2] - pi[2] * pi[2]);
    const double si = 2.0 * (pr[0] * pi[4] + pi[0] * pr[4]) - 2.0 * (pr[1] * pi[3] + pi[1] * pr[3]) +
                      2.0 * pr[2] * pi[2];
    v[8] = 0.5 * (g0 * n * n + g1 * (Fx * Fx + Fy * Fy + Fz * Fz) + g2 * (sr * sr + si * si) / 5.0);
    // external and chemical potential energy density (V + mu) n
    if (pot || mu != 0.0) v[8] += ((pot ? pot[d.psi_off / 5 + r.s] : 0.0) + mu) * n;
  }
  block_sum_store(v, part + (int64_t)blockIdx.x * kNObs);
}

// One block per instance: its observables record, every sum in a fixed order.
//   rec[i][0..9]  observable sums (kNObs), rec[i][10..11] overlap sums,
//   rec[i][12]    reference qubit-norm sum, rec[i][13] step count,
//   rec[i][14]    flags (1: overlap valid, 2: reference valid), rec[i][15] = 0.
__global__ __launch_bounds__(kChunk) void k_reduce_record(LaunchGeom g, const double* __restrict__ part,
                                                         const double* __restrict__ ovpart,
                                                         const double* __restrict__ ref,
                                                         double* __restrict__ rec, double step) {
  __shared__ double sums[kNObs], ovs[kNObs];
  const InstDesc d = g.inst[blockIdx.x];
  double v[kNObs];
#pragma unroll
  for (int k = 0; k < kNObs; ++k) v[k] = 0.0;
  for (int c = threadIdx.x; c < d.nchunks; c += kChunk) {
    const double* p = part + (int64_t)(d.chunk_begin + c) * kNObs;
#pragma unroll
    for (int k = 0; k < kNObs; ++k) v[k] += p[k];
  }
  block_sum_store(v, sums);
  __syncthreads();   // block_sum_store's own LDS is reused below
#pragma unroll
  for (int k = 0; k < kNObs; ++k) v[k] = 0.0;
  if (ovpart) {
    const int nt = d.ntx * d.nty * d.nz;
    for (int t = threadIdx.x; t < nt; t += kChunk) {
      v[0] += ovpart[2 * (d.tile_begin + t)];
      v[1] += ovpart[2 * (d.tile_begin + t) + 1];
    }
  }
  block_sum_store(v, ovs);
  __syncthreads();
  double* r = rec + (int64_t)blockIdx.x * kRecord;
  const int k = threadIdx.x;
  if (k < kNObs) r[k] = sums[k];
  else if (k < kNObs + 2) r[k] = ovs[k - kNObs];
  else if (k == kNObs + 2) r[k] = ref ? ref[(int64_t)blockIdx.x * kRecord] : 0.0;
  else if (k == kNObs + 3) r[k] = step;
  else if (k == kNObs + 4) r[k] = (ovpart ? 1.0 : 0.0) + (ref ? 2.0 : 0.0);
  else if (k < kRecord) r[k] = 0.0;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <typename T>
static Angles<T> angles(double a, double b, double c) {
  return Angles<T>{T(a), T(b), T(c)};
}

template <typename T>
static StepArgs<T> step_args(const void* in, void* out, const LaunchGeom& g, double tg0, double tg1,
                             double tg25, double full_factor, const ExtPot& ext, double* ovpart, int steps,
                             int rows, bool plain, bool overlap) {
  StepArgs<T> A;
  A.in = (const cx<T>*)in;
  A.out = (cx<T>*)out;
  A.inst = g.inst;
  A.tile2inst = g.tile2inst;
  A.ovpart = ovpart;
  A.ang = angles<T>(tg0, tg1, tg25);
  A.ang_full = angles<T>(full_factor * tg0, full_factor * tg1, full_factor * tg25);
  A.pot = ext.V;
  A.mu = ext.mu;
  A.th_ext = T(plain ? full_factor * ext.theta : ext.theta);
  A.prev = (const cx<T>*)in;
  A.zpass = 0;
  A.plain_u = 1;
  A.ntiles = g.ntiles;
  A.steps = steps;
  A.tile_rows = rows;
  A.plain = plain ? 1 : 0;
  A.overlap = overlap ? 1 : 0;
  return A;
}

// Launch `kernel`; with events, the dispatch packet stamps them at kernel start and end.
template <typename K, typename A>
static void launch_timed(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t st, hipEvent_t ev0,
                         hipEvent_t ev1, A args) {
  if (ev0 || ev1)
    hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, st, ev0, ev1, 0u, args);
  else
    hipLaunchKernelGGL(kernel, grid, block, lds, st, args);
}

hipError_t launch_step1d(int dtype, int steps, int split, bool plain, bool overlap, const void* in, void* out,
                         const LaunchGeom& g, double tg0, double tg1, double tg25, const ExtPot& ext,
                         double* ovpart, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (g.ntiles == 0) return hipSuccess;
  static_assert(kLaneTile == kLaneTileSites, "two-lane tile size");
  const int tile = split == 2 ? kLaneTile : kLanes;
  if (split < 0 || split > 2 || steps < 1 || 8 * steps >= tile)
    return hipErrorInvalidValue;
  // the plain split's single U uses theta = eps^2 = 4x the interleaved 1D angle
  const bool xt = ext.on();
  if (split == 2) {
    const dim3 grid((g.ntiles + 3) / 4), block(256);
    if (dtype == 0) {
      const auto args = step_args<float>(in, out, g, tg0, tg1, tg25, 4.0, ext, ovpart, steps, 0, plain, overlap);
      if (xt) launch_timed(k_step1d_lanes<float, true>, grid, block, 0, st, ev0, ev1, args);
      else launch_timed(k_step1d_lanes<float, false>, grid, block, 0, st, ev0, ev1, args);
    } else {
      const auto args = step_args<double>(in, out, g, tg0, tg1, tg25, 4.0, ext, ovpart, steps, 0, plain, overlap);
      if (xt) launch_timed(k_step1d_lanes<double, true>, grid, block, 0, st, ev0, ev1, args);
      else launch_timed(k_step1d_lanes<double, false>, grid, block, 0, st, ev0, ev1, args);
    }
    return hipGetLastError();
  }
  if (split == 1) {
    const dim3 grid((g.ntiles + kPairTiles - 1) / kPairTiles), block(kLanes * kPairWaves);
    if (dtype == 0) {
      const auto args = step_args<float>(in, out, g, tg0, tg1, tg25, 4.0, ext, ovpart, steps, 0, plain, overlap);
      if (xt) launch_timed(k_step1d_pair<float, true>, grid, block, 0, st, ev0, ev1, args);
      else launch_timed(k_step1d_pair<float, false>, grid, block, 0, st, ev0, ev1, args);
    } else {
      const auto args = step_args<double>(in, out, g, tg0, tg1, tg25, 4.0, ext, ovpart, steps, 0, plain, overlap);
      if (xt) launch_timed(k_step1d_pair<double, true>, grid, block, 0, st, ev0, ev1, args);
      else launch_timed(k_step1d_pair<double, false>, grid, block, 0, st, ev0, ev1, args);
    }
    return hipGetLastError();
  }
  const dim3 grid((g.ntiles + 3) / 4), block(256);
  if (dtype == 0) {
    const auto args = step_args<float>(in, out, g, tg0, tg1, tg25, 4.0, ext, ovpart, steps, 0, plain, overlap);
    if (xt) launch_timed(k_step1d<float, true>, grid, block, 0, st, ev0, ev1, args);
    else launch_timed(k_step1d<float, false>, grid, block, 0, st, ev0, ev1, args);
  } else {
    const auto args = step_args<double>(in, out, g, tg0, tg1, tg25, 4.0, ext, ovpart, steps, 0, plain, overlap);
    if (xt) launch_timed(k_step1d<double, true>, grid, block, 0, st, ev0, ev1, args);
    else launch_timed(k_step1d<double, false>, grid, block, 0, st, ev0, ev1, args);
  }
  return hipGetLastError();
}

template <typename T, bool kExt, int kPart>
static void launch_step2d_k(int ntiles, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, const StepArgs<T>& args) {
  const dim3 grid((ntiles + k2DWaves - 1) / k2DWaves), block(64 * k2DWaves);
  const size_t lds = sizeof(cx<T>) * stages_of<kPart>() * kSlotsPerStage * kLanes * k2DWaves;
  launch_timed(k_step2d<T, kExt, kPart>, grid, block, lds, st, ev0, ev1, args);
}

template <typename T>
static hipError_t launch_step2d_t(bool plain, bool overlap, int tile_rows, bool zpass, bool plain_u, int part,
                                  double full_factor, const void* in, void* out, const void* prev,
                                  const LaunchGeom& g, double tg0, double tg1, double tg25, const ExtPot& ext,
                                  double* ovpart, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const int ntiles = zpass ? g.ntiles_z : g.ntiles;
  if (ntiles == 0) return hipSuccess;
  auto args = step_args<T>(in, out, g, tg0, tg1, tg25, full_factor, ext, ovpart, 1, tile_rows, plain, overlap);
  args.prev = (const cx<T>*)prev;
  args.zpass = zpass ? 1 : 0;
  args.plain_u = plain_u ? 1 : 0;
  if (zpass) {
    args.tile2inst = g.tile2inst_z;
    args.ntiles = g.ntiles_z;
  }
  if (ext.on()) {
    if (part == kYFirst) launch_step2d_k<T, true, kYFirst>(ntiles, st, ev0, ev1, args);
    else if (part == kYSecond) launch_step2d_k<T, true, kYSecond>(ntiles, st, ev0, ev1, args);
    else launch_step2d_k<T, true, kWhole>(ntiles, st, ev0, ev1, args);
  } else {
    if (part == kYFirst) launch_step2d_k<T, false, kYFirst>(ntiles, st, ev0, ev1, args);
    else if (part == kYSecond) launch_step2d_k<T, false, kYSecond>(ntiles, st, ev0, ev1, args);
    else launch_step2d_k<T, false, kWhole>(ntiles, st, ev0, ev1, args);
  }
  return hipGetLastError();
}

hipError_t launch_step2d(int dtype, bool plain, bool overlap, int tile_rows, bool zpass, bool plain_u, int part,
                         double full_factor, const void* in, void* out, const void* prev, const LaunchGeom& g,
                         double tg0, double tg1, double tg25, const ExtPot& ext, double* ovpart,
                         hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (tile_rows < 1 || part < kWhole || part > kYSecond) return hipErrorInvalidValue;
  if (dtype == 0)
    return launch_step2d_t<float>(plain, overlap, tile_rows, zpass, plain_u, part, full_factor, in, out, prev, g,
                                  tg0, tg1, tg25, ext, ovpart, st, ev0, ev1);
  return launch_step2d_t<double>(plain, overlap, tile_rows, zpass, plain_u, part, full_factor, in, out, prev, g,
                                 tg0, tg1, tg25, ext, ovpart, st, ev0, ev1);
}

#define QLG_ELEMWISE(NAME, KERNEL, SRC_T, DST_T)                                                    \
  hipError_t NAME(int dtype, SRC_T src, DST_T dst, const LaunchGeom& g, hipStream_t st) {           \
    if (g.nchunks == 0) return hipSuccess;                                                          \
    if (dtype == 0)                                                                                 \
      hipLaunchKernelGGL(KERNEL<float>, dim3(g.nchunks), dim3(kChunk), 0, st, (const cx<float>*)src, \
                         (cx<float>*)dst, g);                                                       \
    else                                                                                            \
      hipLaunchKernelGGL(KERNEL<double>, dim3(g.nchunks), dim3(kChunk), 0, st,                      \
                         (const cx<double>*)src, (cx<double>*)dst, g);                              \
    return hipGetLastError();                                                                       \
  }

QLG_ELEMWISE(launch_set_psi, k_set_psi, const void*, void*)
QLG_ELEMWISE(launch_get_psi, k_get_psi, const void*, void*)
QLG_ELEMWISE(launch_set_qubits, k_set_qubits, const void*, void*)
QLG_ELEMWISE(launch_get_qubits, k_get_qubits, const void*, void*)

hipError_t launch_observables(int dtype, int ndim, const void* state, const LaunchGeom& g, double g0,
                              double g1, double g2, const ExtPot& ext, double* part, hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_observables<float>, dim3(g.nchunks), dim3(kChunk), 0, st, (const cx<float>*)state,
                       g, ndim, g0, g1, g2, ext.V, ext.mu, part);
  else
    hipLaunchKernelGGL(k_observables<double>, dim3(g.nchunks), dim3(kChunk), 0, st,
                       (const cx<double>*)state, g, ndim, g0, g1, g2, ext.V, ext.mu, part);
  return hipGetLastError();
}

hipError_t launch_record(const LaunchGeom& g, const double* part, const double* ovpart, const double* ref,
                         double* rec, int64_t step, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_record, dim3(g.nbatch), dim3(kChunk), 0, st, g, part, ovpart, ref, rec,
                     (double)step);
  return hipGetLastError();
}

}  // namespace qlg
