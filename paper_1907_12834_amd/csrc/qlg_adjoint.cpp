// Adjoint entry points of include/qlg.h: checkpointed forward recording, the
// objective cotangents and the reverse sweep.
//
// Reverse sweep over a recorded run of nsteps with a checkpoint every K steps:
//   for each segment, last to first:
//     recompute, from the segment's checkpoint, the input of every self-interaction substep of
//     its steps (a chain of per-substep kernels, the four x substeps of a step in one);
//     for each step of the segment, last to first, and each substep k, last to first:
//       lambda <- I'_k^H lambda          (exact inverse of the unitary kinetic factor)
//       lambda <- (dU/dz)^H lambda       (FP64 Jacobian at the recomputed substep input)
//   (plain split: one U with theta = eps^2 before the I' list, so only the step input is needed.)
// With two record buffers the recompute of the segment before runs on the context's second
// stream while the sweep pulls lambda back through the current one, its steps issued in step
// with the sweep's.  dL/dg accumulates in FP64
// on the device in a fixed order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "qlg_adjoint.hpp"
#include "qlg_adjoint_kernels.hpp"

namespace {

struct Sizes {
  size_t copy = 0;     // bytes of one padded state copy (forward dtype)
  size_t lam = 0;      // bytes of one padded complex128 cotangent
  int64_t nck = 0;     // checkpoints
  int nsub = 4;        // substeps per step
  int nrec = 4;        // recorded self-interaction inputs per step (nsub, or 1 for the plain split)
  int64_t nchunks = 0; // 256-site chunks of the per-site kernels
  int64_t nx4 = 0;     // wavefronts of the fused x substeps (56 columns of one row each)
  int64_t nparts = 0;  // dg partials (3 doubles each) of one step's reverse sweep
  int64_t part_steps = 1;  // steps whose dg partials are kept before they are summed
  size_t off_zrec = 0, off_y = 0, off_lam = 0, off_part = 0, off_xpre = 0, off_acc = 0, off_red = 0;
  size_t off_zrec2 = 0;  // the second record buffer: the end of the workspace without it
  size_t work = 0;
};

size_t up256(size_t v) { return (v + 255) / 256 * 256; }

// dg partials per chunk of the fused per-site substep kernel (one per wavefront)
constexpr int64_t kSubAdjParts = qlg::kChunk / qlg::kLanes;

// wavefronts of k_adj_x4: ceil(nx / 56) per row of each instance
int64_t adjoint_x4_waves(const qlg_params* p) {
  int64_t n = 0;
  for (int i = 0; i < p->nbatch; ++i) {
    const int64_t ny = p->ndim >= 2 ? p->ny[i] : 1, nz = p->ndim == 3 ? p->nz[i] : 1;
    n += (p->nx[i] + qlg::kValid2D - 1) / qlg::kValid2D * ny * nz;
  }
  return n;
}

int64_t adjoint_chunks(const qlg_params* p) {
  int64_t n = 0;
  for (int i = 0; i < p->nbatch; ++i) {
    const int64_t ny = p->ndim >= 2 ? p->ny[i] : 1, nz = p->ndim == 3 ? p->nz[i] : 1;
    n += (p->nx[i] * ny * nz + qlg::kChunk - 1) / qlg::kChunk;
  }
  return n;
}

qlg_status sizes_for(const qlg_params* p, int64_t nsteps, int32_t K, Sizes* s) {
  if (nsteps < 0 || K < 1) return QLG_ERR_ARG;
  size_t state_bytes = 0, scratch_bytes = 0;
  qlg_status st = qlg_query_sizes(p, &state_bytes, &scratch_bytes);
  if (st) return st;
  const size_t eb = p->dtype == QLG_C64 ? 8 : 16;
  s->copy = state_bytes / 2;
  s->lam = s->copy / eb * 16;
  s->nck = (nsteps + K - 1) / K;
  s->nsub = 4 * p->ndim;
  s->nrec = p->split == QLG_SPLIT_PLAIN ? 1 : s->nsub;
  // chunks of the per-site kernels: ceil(sites / 256) per instance, as the context's layout
  // counts them (every extent of the instance, 1D to 3D)
  const int64_t nchunks = adjoint_chunks(p);
  s->nchunks = nchunks;
  s->nx4 = adjoint_x4_waves(p);
  // a step's dg partials: per chunk for the substeps of the plain split, per wavefront (four per
  // chunk) for the z and y substeps of the interleaved split, then per wavefront for its four
  // fused x substeps
  s->nparts = p->split == QLG_SPLIT_PLAIN ? s->nsub * nchunks
                                         : (s->nsub - 4) * kSubAdjParts * nchunks + s->nx4;
  size_t o = 0;
  // inputs of every self-interaction of one checkpoint segment: [K][nrec] state copies
  s->off_zrec = o;  o += up256((size_t)K * (size_t)s->nrec * s->copy);
  s->off_y = o;     o += up256(2 * s->copy);   // ping-pong of the forward chain
  s->off_lam = o;   o += up256(2 * s->lam);
  // dg partials: [part_steps][nparts][3], a segment's steps for the interleaved split (summed once
  // per segment), one step for the plain split (summed per step)
  s->part_steps = p->split == QLG_SPLIT_PLAIN ? 1 : K;
  s->off_part = o;
  o += up256(sizeof(double) * 3 * (size_t)s->part_steps * (size_t)std::max<int64_t>(s->nparts, 1));
  s->off_xpre = o;  o += up256(sizeof(int) * ((size_t)p->nbatch + 1));   // k_adj_x4's instance prefix
  s->off_acc = o;   o += up256(sizeof(double) * 4);
  s->off_red = o;   o += up256(sizeof(double) * 3 * (size_t)qlg::kDgBlocks);   // the segment sum's blocks
  // a second [K][nrec] record buffer, last, so that the next segment's inputs can be recomputed
  // while the reverse sweep reads the current one's
  s->off_zrec2 = o; o += up256((size_t)K * (size_t)s->nrec * s->copy);
  s->work = o;
  return QLG_OK;
}

}  // namespace

extern "C" {

qlg_status qlg_adjoint_query(const qlg_params* params, int64_t nsteps, int32_t checkpoint_every,
                             size_t* ckpt_bytes, size_t* work_bytes) {
  if (!ckpt_bytes || !work_bytes) return QLG_ERR_ARG;
  Sizes s;
  qlg_status st = sizes_for(params, nsteps, checkpoint_every, &s);
  if (st) return st;
  *ckpt_bytes = (size_t)s.nck * s.copy;
  *work_bytes = s.work;
  return QLG_OK;
}

qlg_status qlg_forward_record(qlg_ctx* ctx, int64_t nsteps, int32_t K, void* ckpt_dev, size_t ckpt_bytes) {
  if (!ctx) return QLG_ERR_ARG;
  if (qlg::ctx_broken(ctx)) return QLG_ERR_STATE;
  qlg::CtxView v = qlg::ctx_view(ctx);
  Sizes s;
  qlg_status st = sizes_for(v.p, nsteps, K, &s);
  if (st) return qlg::ctx_fail(ctx, st, "bad nsteps or checkpoint_every");
  if (s.nck > 0 && (!ckpt_dev || ckpt_bytes < (size_t)s.nck * s.copy))
    return qlg::ctx_fail(ctx, QLG_ERR_ARG, "checkpoint buffer missing or too small");
  for (int64_t j = 0; j < nsteps; j += K) {
    v = qlg::ctx_view(ctx);
    const char* cur = v.state + (size_t)v.cur * s.copy;
    hipError_t e = hipMemcpyAsync((char*)ckpt_dev + (size_t)(j / K) * s.copy, cur, s.copy,
                                  hipMemcpyDeviceToDevice, v.stream);
    if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "checkpoint copy");
    st = qlg::ctx_step(ctx, std::min<int64_t>(K, nsteps - j));
    if (st) return st;
  }
  return QLG_OK;
}

qlg_status qlg_objective_grad(qlg_ctx* ctx, int32_t kind, const void* target_dev, void* lambda_dev,
                              double* value_host, double* dg_host) {
  if (!ctx) return QLG_ERR_ARG;
  if (qlg::ctx_broken(ctx)) return QLG_ERR_STATE;
  if (!lambda_dev || !value_host) return qlg::ctx_fail(ctx, QLG_ERR_ARG, "lambda or value pointer is NULL");
  if (kind != 0 && kind != 1) return qlg::ctx_fail(ctx, QLG_ERR_ARG, "kind must be 0 (energy) or 1 (fidelity)");
  if (kind == 1 && !target_dev) return qlg::ctx_fail(ctx, QLG_ERR_ARG, "fidelity needs a target");
  const qlg::CtxView v = qlg::ctx_view(ctx);
  const qlg_params& p = *v.p;
  const void* cur = v.state + (size_t)v.cur * v.elems_per_copy * v.elem_bytes;
  const int nc = v.geom.nchunks, nb = v.geom.nbatch;
  const double meas = std::pow(p.eps, p.ndim);
  hipError_t e;
  if (kind == 0) {
    e = qlg::launch_energy_grad(p.dtype, p.ndim, cur, lambda_dev, v.geom, p.eps, p.g0, p.g1, p.g2, v.ext, v.part,
                                v.stream);
    if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "energy gradient kernel");
    std::vector<double> part((size_t)nc * 6);
    e = hipMemcpyAsync(part.data(), v.part, part.size() * 8, hipMemcpyDeviceToHost, v.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(v.stream);
    if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "copy energy partials");
    double tot[4] = {0, 0, 0, 0};
    for (int c = 0; c < nc; ++c)
      for (int k = 0; k < 4; ++k) tot[k] += part[(size_t)6 * c + k];
    *value_host = tot[0];
    if (dg_host) { dg_host[0] = tot[1]; dg_host[1] = tot[2]; dg_host[2] = tot[3]; }
  } else {
    e = qlg::launch_fidelity_grad(p.dtype, cur, target_dev, lambda_dev, v.geom, meas, v.part, v.res, v.stream);
    if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "fidelity gradient kernels");
    std::vector<double> ov((size_t)nb * 3);
    e = hipMemcpyAsync(ov.data(), v.res, ov.size() * 8, hipMemcpyDeviceToHost, v.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(v.stream);
    if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "copy overlaps");
    double tot = 0.0;
    for (int i = 0; i < nb; ++i) tot += ov[3 * i] * ov[3 * i] + ov[3 * i + 1] * ov[3 * i + 1];
    *value_host = tot;
    if (dg_host) { dg_host[0] = dg_host[1] = dg_host[2] = 0.0; }
  }
  for (double x : {*value_host})
    if (!std::isfinite(x)) return qlg::ctx_fail(ctx, QLG_ERR_NUMERIC, "objective is not finite");
  return QLG_OK;
}

qlg_status qlg_adjoint_step(qlg_ctx* ctx, int64_t nsteps, int32_t K, const void* ckpt_dev, void* lambda_dev,
                            void* work_dev, size_t work_bytes, double* dg_host) {
  if (!ctx) return QLG_ERR_ARG;
  if (qlg::ctx_broken(ctx)) return QLG_ERR_STATE;
  const qlg::CtxView v = qlg::ctx_view(ctx);
  const qlg_params& p = *v.p;
  Sizes s;
  qlg_status st = sizes_for(v.p, nsteps, K, &s);
  if (st) return qlg::ctx_fail(ctx, st, "bad nsteps or checkpoint_every");
  if (!lambda_dev) return qlg::ctx_fail(ctx, QLG_ERR_ARG, "lambda is NULL");
  if (nsteps == 0) return QLG_OK;
  if (!ckpt_dev || !work_dev) return qlg::ctx_fail(ctx, QLG_ERR_ARG, "checkpoint or work buffer is NULL");
  if (work_bytes < s.off_zrec2) return qlg::ctx_fail(ctx, QLG_ERR_ARG, "work buffer too small");
  // with the second record buffer, the recompute of segment i - 1 runs on the context's second
  // stream while the reverse sweep of segment i runs on its stream
  const bool overlap = work_bytes >= s.work && s.nck > 1;
  // every per-chunk substep kernel writes 3 partials per chunk of the context's layout, the fused x
  // kernel 3 per wavefront; the workspace region between off_part and off_xpre must hold a step's
  const bool plain = p.split == QLG_SPLIT_PLAIN;
  const int64_t nparts_ctx = plain ? (int64_t)s.nsub * v.geom.nchunks
                                   : (int64_t)(s.nsub - 4) * kSubAdjParts * v.geom.nchunks + s.nx4;
  if (v.geom.nchunks != s.nchunks ||
      (size_t)3 * (size_t)s.part_steps * std::max<int64_t>(nparts_ctx, 1) * sizeof(double) > s.off_xpre - s.off_part)
    return qlg::ctx_fail(ctx, QLG_ERR_ARG, "adjoint partials exceed their workspace region");
  if (((uintptr_t)work_dev & 255) || ((uintptr_t)ckpt_dev & 255))
    return qlg::ctx_fail(ctx, QLG_ERR_ARG, "buffers must be 256-byte aligned");

  char* W = (char*)work_dev;
  // zrec[buf][j][r]: input of self-interaction r of step j of a segment
  char* zrec[2] = {W + s.off_zrec, W + s.off_zrec2};
  char* ybuf[2] = {W + s.off_y, W + s.off_y + s.copy};
  char* lam[2] = {W + s.off_lam, W + s.off_lam + s.lam};
  double* part = (double*)(W + s.off_part);
  double* acc = (double*)(W + s.off_acc);
  double* red = (double*)(W + s.off_red);
  const qlg::LaunchGeom& g = v.geom;
  const hipStream_t str = v.stream;
  const int nd = p.ndim, dt = p.dtype, nsub = s.nsub, nrec = s.nrec;
  const int nchunks = g.nchunks;
  int* xpre = (int*)(W + s.off_xpre);
  const double theta = p.eps * p.eps / (4.0 * nd);
  const double theta_u = plain ? p.eps * p.eps : theta;
  // substep k of a step acts along z, y, x in that order (the last axis of each dimension first)
  auto axis_of = [&](int k) { return nd - 1 - k / 4; };
  auto qb_of = [&](int k) { return (k % 4) < 2 ? 1 : 0; };
  auto zbuf = [&](int b, int64_t j, int r) { return zrec[b] + ((size_t)j * nrec + r) * s.copy; };
  auto seg_steps = [&](int64_t seg) { return (int)std::min<int64_t>(K, nsteps - seg * K); };

  // Forward chain of segment seg from its checkpoint into record buffer b: substep k of step j
  // is "I'_{k-1} then U_k" (the I' of the previous substep, none for the first one), recording
  // every U input.  A chain is issued in ranges of steps, in order: chain_to(c, j1, q) issues
  // steps c.j .. j1 - 1 on stream q; src and yb carry the state between the calls.
  struct Chain {
    int64_t seg;
    int b;
    const void* src;
    int yb;
    int j;
  };
  auto chain_begin = [&](int64_t seg, int b) { return Chain{seg, b, (const char*)ckpt_dev + (size_t)seg * s.copy, 0, 0}; };
  auto chain_to = [&](Chain& c, int j1, hipStream_t q) -> hipError_t {
    const int n_in = seg_steps(c.seg);
    const int b = c.b;
    hipError_t e = hipSuccess;
    if (!plain) {
      // interleaved split: link (0, 0) alone, then per step the links (j, 1 .. nsub - 4) one
      // launch each and the four links that apply x factors, (j, nsub - 3 .. nsub - 1) and
      // (j + 1, 0), in one launch (three in the segment's last step)
      const double tg0 = theta_u * p.g0, tg1 = theta_u * p.g1, tg25 = theta_u * p.g2 / 5.0;
      if (c.j == 0 && j1 > 0) {
        e = qlg::launch_chain(dt, c.src, ybuf[c.yb], zbuf(b, 0, 0), g, -1, 0, true, tg0, tg1, tg25, v.ext, theta_u,
                              q);
        c.src = ybuf[c.yb];
        c.yb ^= 1;
      }
      for (; c.j < j1 && e == hipSuccess; ++c.j) {
        const int j = c.j;
        for (int k = 1; k <= nsub - 4 && e == hipSuccess; ++k) {
          e = qlg::launch_chain(dt, c.src, ybuf[c.yb], zbuf(b, j, k), g, axis_of(k - 1), qb_of(k - 1), true, tg0,
                                tg1, tg25, v.ext, theta_u, q);
          c.src = ybuf[c.yb];
          c.yb ^= 1;
        }
        if (e != hipSuccess) break;
        void* const r[4] = {zbuf(b, j, nsub - 3), zbuf(b, j, nsub - 2), zbuf(b, j, nsub - 1),
                            j + 1 < n_in ? zbuf(b, j + 1, 0) : nullptr};
        e = qlg::launch_chain_x4(dt, c.src, ybuf[c.yb], r, g, xpre, (int)s.nx4, tg0, tg1, tg25, v.ext, theta_u, q);
        c.src = ybuf[c.yb];
        c.yb ^= 1;
      }
      return e;
    }
    for (; c.j < j1; ++c.j) {
      const int j = c.j;
      for (int k = 0; k < nsub; ++k) {
        const int kp = k == 0 ? nsub - 1 : k - 1;
        const bool first = j == 0 && k == 0;
        const bool has_u = k == 0;
        if (j == n_in - 1 && k > 0) break;   // later links feed nothing recorded
        e = qlg::launch_chain(dt, c.src, ybuf[c.yb], has_u ? zbuf(b, j, 0) : nullptr, g, first ? -1 : axis_of(kp),
                              qb_of(kp), has_u, theta_u * p.g0, theta_u * p.g1, theta_u * p.g2 / 5.0, v.ext,
                              theta_u, q);
        if (e != hipSuccess) return e;
        c.src = ybuf[c.yb];
        c.yb ^= 1;
      }
    }
    return e;
  };
  auto record_segment = [&](int64_t seg, int b, hipStream_t q) -> hipError_t {
    Chain c = chain_begin(seg, b);
    return chain_to(c, seg_steps(seg), q);
  };

  hipError_t e = qlg::launch_zero(acc, 4, str);
  if (e == hipSuccess) e = qlg::launch_lam_layout(true, lambda_dev, lam[0], g, str);
  if (e == hipSuccess && !plain) e = qlg::launch_x4_prefix(g, xpre, str);
  if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "adjoint setup");
  hipStream_t aux = nullptr;
  hipEvent_t* ev = nullptr;   // [0], [1]: records of buffer 0, 1 ready; [2]: a sweep done; [3]: setup done
  if (overlap) {
    e = qlg::ctx_aux(ctx, &aux, &ev);
    if (e == hipSuccess) e = hipEventRecord(ev[3], str);
    // the recompute reads xpre and the checkpoints, written on the context's stream
    if (e == hipSuccess) e = hipStreamWaitEvent(aux, ev[3], 0);
    if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "adjoint second stream");
  }
  int lc = 0;
  const int64_t nseg = s.nck;
  if (overlap) {
    e = record_segment(nseg - 1, 0, aux);
    if (e == hipSuccess) e = hipEventRecord(ev[0], aux);
    if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "adjoint forward recompute");
  }
  for (int64_t seg = nseg - 1; seg >= 0; --seg) {
    const int n_in = seg_steps(seg);
    int b = 0;
    // the next segment's chain, issued step by step with this segment's sweep (below), so that
    // both streams hold work whatever the pace of the host's launches
    const bool rec_next = overlap && seg > 0;
    Chain nc{};
    if (overlap) {
      b = (int)((nseg - 1 - seg) & 1);
      if (rec_next) {
        // the next segment's records go to the other buffer, once the sweep that read it ended
        if (seg + 1 < nseg) e = hipStreamWaitEvent(aux, ev[2], 0);
        if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "adjoint stream order");
        nc = chain_begin(seg - 1, 1 - b);
      }
      e = hipStreamWaitEvent(str, ev[b], 0);
      if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "adjoint stream order");
    } else {
      e = record_segment(seg, 0, str);
      if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "adjoint forward recompute");
    }
    for (int j = n_in - 1; j >= 0; --j) {
      double* pj = part + (size_t)3 * (plain ? 0 : (size_t)j * s.nparts);   // this step's partials
      if (!plain) {
        // the step's last four substeps (along x) in one kernel, their dg partials after those
        // of the nsub - 4 per-chunk substeps
        const void* zx[4] = {zbuf(b, j, nsub - 1), zbuf(b, j, nsub - 2), zbuf(b, j, nsub - 3), zbuf(b, j, nsub - 4)};
        e = qlg::launch_adj_x4(dt, zx, lam[lc], lam[1 - lc], g, xpre, (int)s.nx4, theta_u, p.g0, p.g1, p.g2,
                               v.ext, pj + (size_t)3 * (nsub - 4) * kSubAdjParts * nchunks, str);
        if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "adjoint x substeps kernel");
        lc = 1 - lc;
      }
      for (int k = plain ? nsub - 1 : nsub - 5; k >= 0; --k) {
        if (plain) {
          e = qlg::launch_sub_iprime_adj(lam[lc], lam[1 - lc], g, axis_of(k), qb_of(k), str);
          if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "adjoint kinetic kernel");
        } else {
          // kinetic pull-back and self-interaction VJP of substep k in one kernel
          e = qlg::launch_sub_adj(dt, zbuf(b, j, k), lam[lc], lam[1 - lc], g, axis_of(k), qb_of(k), theta_u, p.g0,
                                  p.g1, p.g2, v.ext, pj + (size_t)3 * k * kSubAdjParts * nchunks, str);
          if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "adjoint substep kernel");
        }
        lc = 1 - lc;
      }
      if (plain) {
        e = qlg::launch_sub_vjp(dt, zbuf(b, j, 0), lam[lc], g, theta_u, p.g0, p.g1, p.g2, v.ext, part, acc, str);
        if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "adjoint self-interaction kernel");
      }
      if (rec_next) {
        // the chain's steps in proportion to the sweep's (all of them with the sweep's last step)
        const int64_t m = seg_steps(seg - 1), done = n_in - j;
        e = chain_to(nc, (int)((m * done + n_in - 1) / n_in), aux);
        if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "adjoint forward recompute");
      }
    }
    if (rec_next) {
      e = hipEventRecord(ev[1 - b], aux);
      if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "adjoint stream order");
    }
    if (!plain) {
      // the segment's dg partials, summed once in a fixed order
      e = qlg::launch_dg_reduce(part, (int64_t)n_in * s.nparts, red, acc, str);
      if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "adjoint parameter-gradient reduction");
    }
    if (overlap && seg > 1) {
      e = hipEventRecord(ev[2], str);   // the sweep of this segment has read buffer b
      if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "adjoint stream order");
    }
  }
  e = qlg::launch_lam_layout(false, lam[lc], lambda_dev, g, str);
  double hacc[4] = {0, 0, 0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(hacc, acc, sizeof hacc, hipMemcpyDeviceToHost, str);
  if (e == hipSuccess) e = hipStreamSynchronize(str);
  if (e != hipSuccess) return qlg::ctx_hip(ctx, e, "adjoint finish");
  if (dg_host)
    for (int k = 0; k < 3; ++k) dg_host[k] += hacc[k];
  if (!std::isfinite(hacc[0]) || !std::isfinite(hacc[1]) || !std::isfinite(hacc[2]))
    return qlg::ctx_fail(ctx, QLG_ERR_NUMERIC, "non-finite parameter gradient");
  return QLG_OK;
}

qlg_status qlg_set_psi_adjoint(qlg_ctx* ctx, const void* lambda_dev, void* dpsi_dev) {
  if (!ctx) return QLG_ERR_ARG;
  if (qlg::ctx_broken(ctx)) return QLG_ERR_STATE;
  if (!lambda_dev || !dpsi_dev) return qlg::ctx_fail(ctx, QLG_ERR_ARG, "lambda or dpsi is NULL");
  if (((uintptr_t)lambda_dev & 15) || ((uintptr_t)dpsi_dev & 15))
    return qlg::ctx_fail(ctx, QLG_ERR_ARG, "lambda and dpsi must be 16-byte aligned");
  const qlg::CtxView v = qlg::ctx_view(ctx);
  return qlg::ctx_hip(ctx, qlg::launch_encode_adj(lambda_dev, dpsi_dev, v.geom, v.stream), "encode adjoint kernel");
}

}  // extern "C"
