// C ABI of libqlg (include/qlg.h): context, validation, layout tables, the
// step schedule, hipGraph replay, kernel timing, observables and autotuning.
#include "../../include/qlg.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "qlg_internal.hpp"
#include "qlg_adjoint.hpp"
#include "qlg_diag.hpp"

using qlg::InstDesc;
using qlg::LaunchGeom;

namespace {

constexpr int64_t kMaxExtent = int64_t(1) << 30;
constexpr int64_t kMaxSites = (int64_t(1) << 31) - 1;
constexpr int kMaxSteps1D = 7;   // 4 * S halo sites per side must leave interior lanes
constexpr int kMaxStepsLanes = 3;   // qubit_split 2: 32-site tiles
constexpr int kTunePairSteps = 4;   // the autotuner tries qubit_split 1 up to here (slower beyond)
constexpr int kMinTileRows = 8, kMaxTileRows = 256;

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

struct Layout {
  std::vector<InstDesc> inst;
  int64_t elems_per_copy = 0;     // complex elements in one state copy
  int64_t psi_elems = 0;
  int32_t nchunks = 0;
  int32_t max_tiles = 0;          // tiles at the densest plan (used to size scratch)
  int32_t max_tiles_z = 0;        // 3D z pass: tiles at the densest plan
};

// tiles of 64 sites (qubit_split 0 and 1) or 32 sites (2), 4 * steps halo sites per side
int tiles_1d(int64_t nx, int steps, int split) {
  const int tv = (split == 2 ? qlg::kLaneTileSites : qlg::kLanes) - 8 * steps;
  return (int)((nx + tv - 1) / tv);
}

void tiles_2d(int64_t nx, int64_t ny, int rows, int* ntx, int* nty) {
  *ntx = (int)((nx + qlg::kValid2D - 1) / qlg::kValid2D);
  *nty = (int)((ny + rows - 1) / rows);
}

// 3D z pass: 64-column tiles (no x halo), bands of `rows` along z
void tiles_z(int64_t nx, int64_t nz, int rows, int* ntx, int* ntz) {
  *ntx = (int)((nx + qlg::kLanes - 1) / qlg::kLanes);
  *ntz = (int)((nz + rows - 1) / rows);
}

qlg_status validate(const qlg_params* p, const char** msg) { return qlg::validate_params(p, msg); }

Layout make_layout(const qlg_params* p) {
  Layout L;
  int64_t off = 0, poff = 0;
  int32_t chunk = 0;
  int32_t maxt = 0;
  for (int i = 0; i < p->nbatch; ++i) {
    InstDesc d{};
    d.nx = (int32_t)p->nx[i];
    d.ny = p->ndim >= 2 ? (int32_t)p->ny[i] : 1;
    d.nz = p->ndim == 3 ? (int32_t)p->nz[i] : 1;
    d.sites = d.nx * d.ny * d.nz;
    d.stride = round_up(d.sites, 64);
    d.off = off;
    d.psi_off = poff;
    d.qb_off = 2 * poff;
    d.chunk_begin = chunk;
    d.nchunks = (d.sites + qlg::kChunk - 1) / qlg::kChunk;
    off += 10 * d.stride;
    poff += 5 * (int64_t)d.sites;
    chunk += d.nchunks;
    if (p->ndim == 1) maxt += std::max(tiles_1d(d.nx, kMaxSteps1D, 0), tiles_1d(d.nx, kMaxStepsLanes, 2));
    else { int a, b; tiles_2d(d.nx, d.ny, kMinTileRows, &a, &b); maxt += a * b * d.nz; }
    if (p->ndim == 3) { int a, b; tiles_z(d.nx, d.nz, kMinTileRows, &a, &b); L.max_tiles_z += a * b * d.ny; }
    L.inst.push_back(d);
  }
  L.elems_per_copy = off;
  L.psi_elems = poff;
  L.nchunks = chunk;
  L.max_tiles = maxt;
  return L;
}

// The caller's scratch buffer: reduction partials and records, then the device tables of
// the launch geometry (instance descriptors, tile and chunk maps), so that the library
// allocates no device memory of its own.
struct ScratchLayout {
  size_t obs_part, obs_res, norm0, ov_part;          // byte offsets of the reductions
  size_t inst, tile2inst, chunk2inst, tile2inst_z;   // byte offsets of the tables
  size_t total;
};

ScratchLayout scratch_layout(const Layout& L, int nbatch) {
  ScratchLayout s;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += (bytes + 255) / 256 * 256; return r; };
  s.obs_part = take(sizeof(double) * qlg::kNObs * (size_t)std::max(L.nchunks, 1));
  s.obs_res = take(sizeof(double) * qlg::kRecord * nbatch);   // one observables record
  s.norm0 = take(sizeof(double) * qlg::kRecord * nbatch);     // record of the state at set time
  s.ov_part = take(sizeof(double) * 2 * (size_t)std::max(L.max_tiles, 1));
  s.inst = take(sizeof(InstDesc) * (size_t)nbatch);
  s.tile2inst = take(sizeof(int32_t) * (size_t)std::max(L.max_tiles, 1));
  s.chunk2inst = take(sizeof(int32_t) * (size_t)std::max(L.nchunks, 1));
  s.tile2inst_z = take(sizeof(int32_t) * (size_t)std::max(L.max_tiles_z, 1));
  s.total = o;
  return s;
}

// Process-wide autotune cache keyed by (arch, dtype, ndim, split, size class).
std::mutex g_tune_mu;
std::map<std::string, qlg_tuning> g_tune_cache;

}  // namespace

// Scratch of the contexts that qlg_init_static creates: their reduction partials and device
// tables (the scratch layout above), in one array per GPU that the process holds until it
// ends.  In host code `scratch` names a host-side stand-in, not device memory: host code
// uses only the address hipGetSymbolAddress returns for it, taken once per device with that
// device current.
static __device__ __align__(256) unsigned char scratch[QLG_STATIC_SCRATCH_BYTES];

namespace {

// Per device: the device address of `scratch`, and whether a live context uses it.
struct StaticScratch {
  char* ptr = nullptr;
  bool in_use = false;
};
std::mutex g_static_mu;
std::map<int, StaticScratch> g_static;

}  // namespace

struct qlg_ctx {
  qlg_params p{};
  std::vector<int64_t> nx, ny, nz;
  Layout L;
  ScratchLayout S{};
  char* state = nullptr;
  size_t state_bytes = 0;
  char* scratch = nullptr;
  size_t scratch_bytes = 0;
  hipStream_t stream = nullptr;
  int cur = 0;
  size_t elem_bytes = 8;
  // device tables (inside the scratch buffer)
  InstDesc* d_inst = nullptr;
  int32_t* d_tile2inst = nullptr;
  int32_t* d_chunk2inst = nullptr;
  int32_t* d_tile2inst_z = nullptr;   // 3D z pass
  int32_t ntiles = 0, ntiles_z = 0;
  qlg_tuning tuning{1, 32, 0, 0};
  qlg::ExtPot ext;               // external potential (caller's device array) and mu
  bool tuned = false;
  int static_dev = -1;            // device whose static scratch this context uses, or -1
  int device = 0;                 // the device current at qlg_init (the buffers' device)
  // bookkeeping
  int64_t step_count = 0;
  bool has_overlap = false;
  bool norm0_valid = false;
  bool broken = false;
  std::string err;
  // graphs keyed by (nsteps, start copy)
  std::map<std::pair<int64_t, int>, hipGraphExec_t> graphs;
  // the adjoint's second stream (default priority) and its events, made on first use
  hipStream_t aux = nullptr;
  hipEvent_t aux_ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev;
  double time_ms = 0.0;          // summed kernel time since timing was enabled
  int64_t time_launches = 0;

  LaunchGeom geom() const {
    LaunchGeom g;
    g.inst = d_inst;
    g.tile2inst = d_tile2inst;
    g.chunk2inst = d_chunk2inst;
    g.tile2inst_z = d_tile2inst_z;
    g.ntiles = ntiles;
    g.ntiles_z = ntiles_z;
    g.nchunks = L.nchunks;
    g.nbatch = p.nbatch;
    return g;
  }
  char* copy(int c) const { return state + (size_t)c * L.elems_per_copy * elem_bytes; }
  double* sc(size_t off) const { return reinterpret_cast<double*>(scratch + off); }
};

namespace {

qlg_status fail(qlg_ctx* c, qlg_status s, const std::string& m) {
  if (c) {
    c->err = m;
    if (s == QLG_ERR_DEVICE) c->broken = true;
  }
  return s;
}

qlg_status hip_check(qlg_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return QLG_OK;
  return fail(c, QLG_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void drop_graphs(qlg_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

// Rebuild the wave-tile tables for the current plan.
qlg_status build_tiles(qlg_ctx* c) {
  std::vector<int32_t> t2i, t2i_z;
  for (int i = 0; i < c->p.nbatch; ++i) {
    InstDesc& d = c->L.inst[i];
    d.tile_begin = (int32_t)t2i.size();
    if (c->p.ndim == 1) {
      d.ntx = tiles_1d(d.nx, c->tuning.steps_per_pass, c->tuning.qubit_split);
      d.nty = 1;
    } else {
      tiles_2d(d.nx, d.ny, c->tuning.tile_rows, &d.ntx, &d.nty);
    }
    for (int64_t k = 0; k < (int64_t)d.ntx * d.nty * d.nz; ++k) t2i.push_back(i);
    if (c->p.ndim == 3) {
      d.tile_begin_z = (int32_t)t2i_z.size();
      tiles_z(d.nx, d.nz, c->tuning.tile_rows, &d.ntx_z, &d.ntz);
      for (int64_t k = 0; k < (int64_t)d.ntx_z * d.ntz * d.ny; ++k) t2i_z.push_back(i);
    }
  }
  if ((int32_t)t2i.size() > c->L.max_tiles || (int32_t)t2i_z.size() > c->L.max_tiles_z)
    return fail(c, QLG_ERR_ARG, "tile table overflow");
  c->ntiles = (int32_t)t2i.size();
  c->ntiles_z = (int32_t)t2i_z.size();
  c->has_overlap = false;   // overlap partials refer to the previous tile layout
  qlg_status s = hip_check(c, hipMemcpyAsync(c->d_inst, c->L.inst.data(), sizeof(InstDesc) * c->L.inst.size(),
                                             hipMemcpyHostToDevice, c->stream), "copy instance table");
  if (s) return s;
  s = hip_check(c, hipMemcpyAsync(c->d_tile2inst, t2i.data(), sizeof(int32_t) * t2i.size(),
                                  hipMemcpyHostToDevice, c->stream), "copy tile table");
  if (s) return s;
  if (!t2i_z.empty()) {
    s = hip_check(c, hipMemcpyAsync(c->d_tile2inst_z, t2i_z.data(), sizeof(int32_t) * t2i_z.size(),
                                    hipMemcpyHostToDevice, c->stream), "copy z tile table");
    if (s) return s;
  }
  // the host vectors must outlive the async copies
  s = hip_check(c, hipStreamSynchronize(c->stream), "sync after table upload");
  drop_graphs(c);
  return s;
}

qlg_status check_ctx(qlg_ctx* c) {
  if (!c) return QLG_ERR_ARG;
  if (c->broken) return QLG_ERR_STATE;
  return QLG_OK;
}

double angle_scale(const qlg_ctx* c) {   // interleaved theta = eps^2 / (4 d)
  return c->p.eps * c->p.eps / (4.0 * c->p.ndim);
}

// Whether one step leaves the state in the copy it started from: a 3D step (its z pass
// from `in` to `out`, its y-x pass back), and a 2D step whose y half is split over two
// launches (the same way).  Otherwise a pass writes the other copy.
bool step_returns(const qlg_ctx* c) {
  return c->p.ndim == 3 || (c->p.ndim == 2 && c->tuning.qubit_split == 1);
}

// One pass of the fused step from `in` to `out` (1D: `steps` steps; 2D: one step).
// 3D, and 2D with the y half split (qubit_split 1): one step as several launches that
// alternate between `in` and `out`, ending in `in`: 3D the z pass (one launch, or two with
// the split) and the y-x pass (one or two), 2D the two halves of the y half, the second
// with the x half; with keep_state (timing runs) every launch reads `in` and writes `out`,
// leaving `in` unchanged.  ev0 / ev1 are stamped at the start of the first and the end of
// the last kernel.
hipError_t launch_pass(qlg_ctx* c, int steps, bool overlap, void* in, void* out, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr, bool keep_state = false) {
  const double th = angle_scale(c);
  const LaunchGeom g = c->geom();
  double* ov = c->sc(c->S.ov_part);
  const bool plain = c->p.split == QLG_SPLIT_PLAIN;
  const double tg0 = th * c->p.g0, tg1 = th * c->p.g1, tg25 = th * c->p.g2 / 5.0;
  qlg::ExtPot ext = c->ext;
  ext.theta = th;
  const int rows = c->tuning.tile_rows;
  const int dt = c->p.dtype;
  if (c->p.ndim == 1)
    return qlg::launch_step1d(dt, steps, c->tuning.qubit_split, plain, overlap, in, out, g, tg0, tg1, tg25, ext,
                              ov, c->stream, ev0, ev1);
  const double ff = c->p.ndim == 2 ? 8.0 : 12.0;
  // A 3D step over four launches overwrites `in` (the state before the step) with its second
  // launch, so a step that records the overlap with that state runs as two launches.  Both
  // forms compute the same numbers: the split stores the state between its launches at its
  // true scale, an exact power-of-two rescaling of the one-launch form's intermediate.
  const bool ysplit = c->tuning.qubit_split == 1 && !(c->p.ndim == 3 && overlap);
  if (c->p.ndim == 2 && !ysplit)
    return qlg::launch_step2d(dt, plain, overlap, rows, false, true, qlg::kWhole, ff, in, out, in, g, tg0, tg1,
                              tg25, ext, ov, c->stream, ev0, ev1);
  // the launches of one step: (z pass, part, applies the plain U, records the overlap)
  struct L { bool zpass; int part; bool plain_u; bool last; };
  L seq[4];
  int n = 0;
  if (c->p.ndim == 3) {
    if (ysplit) {
      seq[n++] = {true, qlg::kYFirst, true, false};
      seq[n++] = {true, qlg::kYSecond, false, false};
    } else {
      seq[n++] = {true, qlg::kWhole, true, false};
    }
  }
  if (ysplit) {
    seq[n++] = {false, qlg::kYFirst, c->p.ndim == 2, false};
    seq[n++] = {false, qlg::kYSecond, false, true};
  } else {
    seq[n++] = {false, qlg::kWhole, false, true};
  }
  void* src = in;
  void* dst = out;
  for (int k = 0; k < n; ++k) {
    const L& l = seq[k];
    hipError_t e = qlg::launch_step2d(dt, plain, l.last && overlap, rows, l.zpass, l.plain_u, l.part, ff, src,
                                      dst, in, g, tg0, tg1, tg25, ext, ov, c->stream, k == 0 ? ev0 : nullptr,
                                      k == n - 1 ? ev1 : nullptr);
    if (e != hipSuccess) return e;
    if (!keep_state) std::swap(src, dst);
  }
  return hipSuccess;
}

// Enqueue nsteps as passes of steps_per_pass (1D) or single steps (2D), ping-ponging
// between the two copies.  The last pass records the overlap partials.
qlg_status enqueue_steps(qlg_ctx* c, int64_t nsteps, int* cur, bool timed) {
  const int S = c->p.ndim == 1 ? c->tuning.steps_per_pass : 1;
  int64_t left = nsteps;
  int64_t launch = 0;
  while (left > 0) {
    const int s = (int)std::min<int64_t>(S, left);
    const bool last = left == s;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed && 2 * (size_t)launch + 1 < c->ev.size()) {
      e0 = c->ev[2 * (size_t)launch];
      e1 = c->ev[2 * (size_t)launch + 1];
    }
    hipError_t e = launch_pass(c, s, last, c->copy(*cur), c->copy(1 - *cur), e0, e1);
    if (e != hipSuccess) return hip_check(c, e, "step kernel launch");
    if (!step_returns(c)) *cur = 1 - *cur;
    left -= s;
    ++launch;
  }
  return QLG_OK;
}

std::string tune_key(const qlg_ctx* c) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop{};
  (void)hipGetDeviceProperties(&prop, dev);
  int64_t sites = 0;
  for (auto& d : c->L.inst) sites += d.sites;
  int sclass = 0;
  while ((int64_t(1) << sclass) < sites) ++sclass;
  char buf[256];
  snprintf(buf, sizeof buf, "%s|%d|%d|%d|%d|%d", prop.gcnArchName, c->p.dtype, c->p.ndim, c->p.split,
           c->p.nbatch > 1 ? 1 : 0, sclass);
  return buf;
}

// A launch plan's range checks for this context (those of qlg_set_tuning): nullptr when valid.
const char* tuning_error(const qlg_ctx* c, const qlg_tuning& n) {
  if (c->p.ndim == 1) {
    if (n.steps_per_pass < 1 || n.steps_per_pass > kMaxSteps1D) return "steps_per_pass must be 1..7 in 1D";
    if (n.qubit_split < 0 || n.qubit_split > 2) return "qubit_split must be 0, 1 or 2";
    if (n.qubit_split == 2 && n.steps_per_pass > kMaxStepsLanes) return "steps_per_pass must be 1..3 with qubit_split 2";
  } else {
    if (n.steps_per_pass != 1) return "steps_per_pass must be 1 in 2D and 3D";
    if (n.qubit_split != 0 && n.qubit_split != 1) return "qubit_split must be 0 or 1 in 2D and 3D";
    if (n.tile_rows < kMinTileRows || n.tile_rows > kMaxTileRows) return "tile_rows must be 8..256";
  }
  return nullptr;
}

// Autotune results that outlive the process: when the environment variable QLG_TUNE_CACHE
// names a file, qlg_autotune appends "key steps_per_pass tile_rows use_graph qubit_split" to
// it, and a new context takes the plan of the last line with its key (a line with a plan
// that is out of range for the context is ignored).  Read before the process-wide cache.
bool tune_file_lookup(const qlg_ctx* c, const std::string& key, qlg_tuning* out) {
  const char* path = std::getenv("QLG_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  bool found = false;
  char k[200];
  qlg_tuning t{};
  while (std::fscanf(f, "%199s %d %d %d %d", k, &t.steps_per_pass, &t.tile_rows, &t.use_graph,
                     &t.qubit_split) == 5)
    if (key == k && !tuning_error(c, t)) { *out = t; found = true; }
  std::fclose(f);
  if (found && c->p.ndim == 1) out->tile_rows = 0;
  if (found) out->use_graph = out->use_graph ? 1 : 0;
  return found;
}

void tune_file_store(const std::string& key, const qlg_tuning& t) {
  const char* path = std::getenv("QLG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %d\n", key.c_str(), t.steps_per_pass, t.tile_rows, t.use_graph, t.qubit_split);
  std::fclose(f);
}

}  // namespace

extern "C" {

int32_t qlg_version(void) { return 10200; }

const char* qlg_status_string(qlg_status s) {
  switch (s) {
    case QLG_OK: return "QLG_OK";
    case QLG_ERR_ARG: return "QLG_ERR_ARG";
    case QLG_ERR_SHAPE: return "QLG_ERR_SHAPE";
    case QLG_ERR_DTYPE: return "QLG_ERR_DTYPE";
    case QLG_ERR_DEVICE: return "QLG_ERR_DEVICE";
    case QLG_ERR_OOM: return "QLG_ERR_OOM";
    case QLG_ERR_STATE: return "QLG_ERR_STATE";
    case QLG_ERR_NUMERIC: return "QLG_ERR_NUMERIC";
  }
  return "QLG_ERR_UNKNOWN";
}

const char* qlg_last_error(const qlg_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

qlg_status qlg_inject_device_error(qlg_ctx* c, const char* reason) {
  qlg_status s = check_ctx(c);
  if (s) return s;
  return fail(c, QLG_ERR_DEVICE, std::string("injected device error: ") + (reason ? reason : ""));
}

qlg_status qlg_query_sizes(const qlg_params* p, size_t* state_bytes, size_t* scratch_bytes) {
  const char* msg = nullptr;
  qlg_status s = validate(p, &msg);
  if (s) return s;
  if (!state_bytes || !scratch_bytes) return QLG_ERR_ARG;
  const Layout L = make_layout(p);
  const size_t eb = p->dtype == QLG_C64 ? 8 : 16;
  *state_bytes = 2 * (size_t)L.elems_per_copy * eb;
  *scratch_bytes = scratch_layout(L, p->nbatch).total;
  return QLG_OK;
}

static qlg_status init_ctx(const qlg_params* p, void* state_dev, size_t state_bytes, void* scratch_dev,
                           size_t scratch_bytes, void* hip_stream, int static_dev, qlg_ctx** out) {
  if (!out) return QLG_ERR_ARG;
  *out = nullptr;
  const char* msg = nullptr;
  qlg_status s = validate(p, &msg);
  if (s) return s;
  if (!state_dev || !scratch_dev) return QLG_ERR_ARG;
  if (((uintptr_t)state_dev & 255) || ((uintptr_t)scratch_dev & 255)) return QLG_ERR_ARG;
  size_t need_state = 0, need_scratch = 0;
  qlg_query_sizes(p, &need_state, &need_scratch);
  if (state_bytes < need_state || scratch_bytes < need_scratch) return QLG_ERR_ARG;

  qlg_ctx* c = new (std::nothrow) qlg_ctx();
  if (!c) return QLG_ERR_OOM;
  c->static_dev = static_dev;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return QLG_ERR_DEVICE;
  }
  c->p = *p;
  c->nx.assign(p->nx, p->nx + p->nbatch);
  if (p->ndim >= 2) c->ny.assign(p->ny, p->ny + p->nbatch);
  else c->ny.assign(p->nbatch, 1);
  if (p->ndim == 3) c->nz.assign(p->nz, p->nz + p->nbatch);
  else c->nz.assign(p->nbatch, 1);
  c->p.nx = c->nx.data();
  c->p.ny = c->ny.data();
  c->p.nz = c->nz.data();
  c->L = make_layout(&c->p);
  c->S = scratch_layout(c->L, p->nbatch);
  c->state = (char*)state_dev;
  c->state_bytes = state_bytes;
  c->scratch = (char*)scratch_dev;
  c->scratch_bytes = scratch_bytes;
  c->stream = (hipStream_t)hip_stream;
  c->elem_bytes = p->dtype == QLG_C64 ? 8 : 16;
  if (p->ndim >= 2) c->tuning = qlg_tuning{1, 32, 0, 0};
  else c->tuning = qlg_tuning{1, 0, 0, 0};

  c->d_inst = reinterpret_cast<InstDesc*>(c->scratch + c->S.inst);
  c->d_tile2inst = reinterpret_cast<int32_t*>(c->scratch + c->S.tile2inst);
  c->d_chunk2inst = reinterpret_cast<int32_t*>(c->scratch + c->S.chunk2inst);
  if (p->ndim == 3) c->d_tile2inst_z = reinterpret_cast<int32_t*>(c->scratch + c->S.tile2inst_z);
  std::vector<int32_t> c2i;
  for (int i = 0; i < p->nbatch; ++i)
    for (int k = 0; k < c->L.inst[i].nchunks; ++k) c2i.push_back(i);
  hipError_t e = hipMemcpy(c->d_chunk2inst, c2i.data(), sizeof(int32_t) * c2i.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    qlg_destroy(c);
    return QLG_ERR_DEVICE;
  }
  {
    const std::string key = tune_key(c);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    qlg_tuning t{};
    if (tune_file_lookup(c, key, &t)) {
      c->tuning = t;
      c->tuned = true;
    } else {
      auto it = g_tune_cache.find(key);
      if (it != g_tune_cache.end()) { c->tuning = it->second; c->tuned = true; }
    }
  }
  s = build_tiles(c);
  if (s) {
    qlg_destroy(c);
    return s;
  }
  *out = c;
  return QLG_OK;
}

qlg_status qlg_init(const qlg_params* p, void* state_dev, size_t state_bytes, void* scratch_dev,
                    size_t scratch_bytes, void* hip_stream, qlg_ctx** out) {
  return init_ctx(p, state_dev, state_bytes, scratch_dev, scratch_bytes, hip_stream, -1, out);
}

qlg_status qlg_init_static(const qlg_params* p, void* state_dev, size_t state_bytes, void* hip_stream,
                           qlg_ctx** out) {
  if (!out) return QLG_ERR_ARG;
  *out = nullptr;
  size_t need_state = 0, need_scratch = 0;
  qlg_status s = qlg_query_sizes(p, &need_state, &need_scratch);
  if (s) return s;
  if (need_scratch > (size_t)QLG_STATIC_SCRATCH_BYTES) return QLG_ERR_ARG;   // lattice too large for it
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return QLG_ERR_DEVICE;
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    StaticScratch& slot = g_static[dev];
    if (slot.in_use) return QLG_ERR_STATE;   // one such context per device at a time
    if (!slot.ptr) {
      void* ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return QLG_ERR_DEVICE;
      slot.ptr = static_cast<char*>(ptr);
    }
    slot.in_use = true;
    base = slot.ptr;
  }
  s = init_ctx(p, state_dev, state_bytes, base, (size_t)QLG_STATIC_SCRATCH_BYTES, hip_stream, dev, out);
  if (s) {
    std::lock_guard<std::mutex> lk(g_static_mu);
    g_static[dev].in_use = false;
  }
  return s;
}

void qlg_destroy(qlg_ctx* c) {
  if (!c) return;
  drop_graphs(c);
  for (auto ev : c->ev) (void)hipEventDestroy(ev);
  if (c->aux) {
    // the adjoint orders every kernel of the second stream before the context's stream's end,
    // but a failed call may have left some queued
    (void)hipStreamSynchronize(c->aux);
    (void)hipStreamDestroy(c->aux);
  }
  for (auto ev : c->aux_ev)
    if (ev) (void)hipEventDestroy(ev);
  if (c->static_dev >= 0) {
    // work still queued on the context's stream may use the array: let it finish first
    (void)hipStreamSynchronize(c->stream);
    std::lock_guard<std::mutex> lk(g_static_mu);
    g_static[c->static_dev].in_use = false;
  }
  delete c;
}

// Enqueue the observables record of the current state into rec (device).
static qlg_status enqueue_record(qlg_ctx* c, double* rec, bool reference) {
  const LaunchGeom g = c->geom();
  hipError_t e = qlg::launch_observables(c->p.dtype, c->p.ndim, c->copy(c->cur), g, c->p.g0, c->p.g1, c->p.g2,
                                         c->ext, c->sc(c->S.obs_part), c->stream);
  if (e != hipSuccess) return hip_check(c, e, "observables kernel");
  const double* ov = (!reference && c->has_overlap) ? c->sc(c->S.ov_part) : nullptr;
  const double* ref = (!reference && c->norm0_valid) ? c->sc(c->S.norm0) : nullptr;
  e = qlg::launch_record(g, c->sc(c->S.obs_part), ov, ref, rec, c->step_count, c->stream);
  return e == hipSuccess ? QLG_OK : hip_check(c, e, "observables record kernel");
}

static qlg_status after_set(qlg_ctx* c) {
  c->step_count = 0;
  c->has_overlap = false;
  // reference record (qubit norm at set time) for the drift check, kept on the device
  qlg_status s = enqueue_record(c, c->sc(c->S.norm0), true);
  if (s) return s;
  c->norm0_valid = true;
  return QLG_OK;
}

qlg_status qlg_set_psi(qlg_ctx* c, const void* psi) {
  qlg_status s = check_ctx(c);
  if (s) return s;
  if (!psi) return fail(c, QLG_ERR_ARG, "psi is NULL");
  hipError_t e = qlg::launch_set_psi(c->p.dtype, psi, c->copy(c->cur), c->geom(), c->stream);
  if (e != hipSuccess) return hip_check(c, e, "set_psi kernel");
  return after_set(c);
}

qlg_status qlg_get_psi(qlg_ctx* c, void* psi) {
  qlg_status s = check_ctx(c);
  if (s) return s;
  if (!psi) return fail(c, QLG_ERR_ARG, "psi is NULL");
  return hip_check(c, qlg::launch_get_psi(c->p.dtype, c->copy(c->cur), psi, c->geom(), c->stream), "get_psi kernel");
}

qlg_status qlg_set_qubits(qlg_ctx* c, const void* qb) {
  qlg_status s = check_ctx(c);
  if (s) return s;
  if (!qb) return fail(c, QLG_ERR_ARG, "qubits is NULL");
  hipError_t e = qlg::launch_set_qubits(c->p.dtype, qb, c->copy(c->cur), c->geom(), c->stream);
  if (e != hipSuccess) return hip_check(c, e, "set_qubits kernel");
  return after_set(c);
}

qlg_status qlg_get_qubits(qlg_ctx* c, void* qb) {
  qlg_status s = check_ctx(c);
  if (s) return s;
  if (!qb) return fail(c, QLG_ERR_ARG, "qubits is NULL");
  return hip_check(c, qlg::launch_get_qubits(c->p.dtype, c->copy(c->cur), qb, c->geom(), c->stream),
                   "get_qubits kernel");
}

qlg_status qlg_set_potential(qlg_ctx* c, const double* V, double mu) {
  qlg_status s = check_ctx(c);
  if (s) return s;
  if (!std::isfinite(mu)) return fail(c, QLG_ERR_ARG, "mu must be finite");
  if (V && (reinterpret_cast<uintptr_t>(V) & 7u)) return fail(c, QLG_ERR_ARG, "V must be 8-byte aligned");
  c->ext.V = V;
  c->ext.mu = mu;
  drop_graphs(c);   // captured launches carry the previous kernel and arguments
  return QLG_OK;
}

qlg_status qlg_fields(qlg_ctx* c, double* n, double* f_par, double* f_perp, double* a00) {
  qlg_status s = check_ctx(c);
  if (s) return s;
  if (!n && !f_par && !f_perp && !a00) return fail(c, QLG_ERR_ARG, "every field output is NULL");
  return hip_check(c, qlg::launch_fields(c->p.dtype, c->copy(c->cur), c->geom(), n, f_par, f_perp, a00, c->stream),
                   "fields kernel");
}

qlg_status qlg_vorticity(qlg_ctx* c, int32_t m_index, double* omega, int32_t* winding) {
  qlg_status s = check_ctx(c);
  if (s) return s;
  if (c->p.ndim < 2) return fail(c, QLG_ERR_SHAPE, "vorticity needs a 2D or 3D lattice");
  if (m_index < 0 || m_index > 4) return fail(c, QLG_ERR_ARG, "m_index must be in 0..4");
  if (!omega && !winding) return fail(c, QLG_ERR_ARG, "omega and winding are both NULL");
  for (const qlg::InstDesc& d : c->L.inst) {
    s = hip_check(c, qlg::launch_vorticity(c->p.dtype, c->p.ndim, c->copy(c->cur), d, m_index, omega, winding,
                                           c->L.psi_elems / 5, c->stream),
                  "vorticity kernel");
    if (s) return s;
  }
  return QLG_OK;
}

qlg_status qlg_find_vortices(qlg_ctx* c, int32_t m_index, int32_t* winding, int32_t* cores, int64_t capacity,
                             int64_t* count) {
  qlg_status s = check_ctx(c);
  if (s) return s;
  if (c->p.ndim < 2) return fail(c, QLG_ERR_SHAPE, "vortex cores need a 2D or 3D lattice");
  if (m_index < 0 || m_index > 4) return fail(c, QLG_ERR_ARG, "m_index must be in 0..4");
  if (!winding || !count) return fail(c, QLG_ERR_ARG, "winding or count is NULL");
  if (capacity < 0 || (capacity > 0 && !cores)) return fail(c, QLG_ERR_ARG, "bad capacity or NULL cores");
  for (const qlg::InstDesc& d : c->L.inst) {
    s = hip_check(c, qlg::launch_vorticity(c->p.dtype, c->p.ndim, c->copy(c->cur), d, m_index, nullptr, winding,
                                           c->L.psi_elems / 5, c->stream),
                  "vorticity kernel");
    if (s) return s;
  }
  // the counts of one chunk per plane family (three in 3D) fit in the kNObs doubles per chunk
  // of the observables' partials
  static_assert(qlg::kNObs >= 3, "core counts need three int64 per chunk");
  int64_t* counts = reinterpret_cast<int64_t*>(c->sc(c->S.obs_part));
  return hip_check(c, qlg::launch_vortex_cores(winding, c->geom(), c->p.ndim, c->L.psi_elems / 5, counts, cores,
                                               capacity, count, c->stream),
                   "vortex core kernels");
}

qlg_status qlg_step(qlg_ctx* c, int64_t nsteps) {
  qlg_status s = check_ctx(c);
  if (s) return s;
  if (nsteps < 0) return fail(c, QLG_ERR_ARG, "nsteps must be >= 0");
  if (nsteps == 0) return QLG_OK;
  const int S = c->p.ndim == 1 ? c->tuning.steps_per_pass : 1;
  const int64_t launches = (nsteps + S - 1) / S;
  if (c->timing) {
    const size_t need = 2 * (size_t)std::min<int64_t>(launches, 4096);
    while (c->ev.size() < need) {
      hipEvent_t ev;
      if (hipEventCreate(&ev) != hipSuccess) break;
      c->ev.push_back(ev);
    }
    int cur = c->cur;
    s = enqueue_steps(c, nsteps, &cur, true);
    if (s) return s;
    c->cur = cur;
    s = hip_check(c, hipStreamSynchronize(c->stream), "sync for timing");
    if (s) return s;
    for (int64_t k = 0; k < launches && 2 * (size_t)k + 1 < c->ev.size(); ++k) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]) == hipSuccess) {
        c->time_ms += ms;
        ++c->time_launches;
      }
    }
  } else if (c->tuning.use_graph && launches > 1) {
    auto key = std::make_pair(nsteps, c->cur);
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
      hipStream_t cap = nullptr;
      hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_check(c, e, "create capture stream");
      hipStream_t saved = c->stream;
      c->stream = cap;
      e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      int cur = c->cur;
      if (e == hipSuccess) s = enqueue_steps(c, nsteps, &cur, false);
      hipGraph_t graph = nullptr;
      hipError_t e2 = hipStreamEndCapture(cap, &graph);
      c->stream = saved;
      (void)hipStreamDestroy(cap);
      if (e != hipSuccess) return hip_check(c, e, "begin capture");
      if (s) { if (graph) (void)hipGraphDestroy(graph); return s; }
      if (e2 != hipSuccess) return hip_check(c, e2, "end capture");
      hipGraphExec_t exec = nullptr;
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return hip_check(c, e, "instantiate graph");
      it = c->graphs.emplace(key, exec).first;
    }
    s = hip_check(c, hipGraphLaunch(it->second, c->stream), "graph launch");
    if (s) return s;
    if (launches % 2 && !step_returns(c)) c->cur = 1 - c->cur;
  } else {
    int cur = c->cur;
    s = enqueue_steps(c, nsteps, &cur, false);
    if (s) return s;
    c->cur = cur;
  }
  c->step_count += nsteps;
  c->has_overlap = true;
  return QLG_OK;
}

// Host decoding of nrec records of nbatch instances; false if any is non-finite
// or drifted.
static bool decode_records(const qlg_ctx* c, const double* rec, int64_t nrec, qlg_obs* out) {
  return qlg::decode_record_values(c->p, rec, nrec, out);
}

qlg_status qlg_observables(qlg_ctx* c, qlg_obs* out) {
  qlg_status s = check_ctx(c);
  if (s) return s;
  if (!out) return fail(c, QLG_ERR_ARG, "out is NULL");
  s = enqueue_record(c, c->sc(c->S.obs_res), false);
  if (s) return s;
  std::vector<double> rec((size_t)c->p.nbatch * qlg::kRecord);
  hipError_t e = hipMemcpyAsync(rec.data(), c->sc(c->S.obs_res), rec.size() * 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_check(c, e, "copy observables");
  if (!decode_records(c, rec.data(), 1, out))
    return fail(c, QLG_ERR_NUMERIC, "non-finite observable or qubit-norm drift above threshold");
  return QLG_OK;
}

qlg_status qlg_record_observables(qlg_ctx* c, double* rec_dev) {
  qlg_status s = check_ctx(c);
  if (s) return s;
  if (!rec_dev) return fail(c, QLG_ERR_ARG, "rec_dev is NULL");
  return enqueue_record(c, rec_dev, false);
}

qlg_status qlg_decode_records(qlg_ctx* c, const double* rec_host, int64_t nrec, qlg_obs* out_host) {
  qlg_status s = check_ctx(c);
  if (s) return s;
  if (nrec < 0) return fail(c, QLG_ERR_ARG, "nrec must be >= 0");
  if (nrec > 0 && (!rec_host || !out_host)) return fail(c, QLG_ERR_ARG, "rec_host or out_host is NULL");
  if (!decode_records(c, rec_host, nrec, out_host))
    return fail(c, QLG_ERR_NUMERIC, "non-finite observable or qubit-norm drift above threshold");
  return QLG_OK;
}

qlg_status qlg_set_tuning(qlg_ctx* c, const qlg_tuning* t) {
  qlg_status s = check_ctx(c);
  if (s) return s;
  if (!t) return fail(c, QLG_ERR_ARG, "tuning is NULL");
  qlg_tuning n = *t;
  if (const char* why = tuning_error(c, n)) return fail(c, QLG_ERR_ARG, why);
  if (c->p.ndim == 1) n.tile_rows = 0;
  n.use_graph = n.use_graph ? 1 : 0;
  c->tuning = n;
  return build_tiles(c);
}

qlg_status qlg_get_tuning(const qlg_ctx* c, qlg_tuning* t) {
  if (!c || !t) return QLG_ERR_ARG;
  if (c->broken) return QLG_ERR_STATE;
  *t = c->tuning;
  return QLG_OK;
}

qlg_status qlg_autotune(qlg_ctx* c) {
  qlg_status s = check_ctx(c);
  if (s) return s;
  // Candidates in order of preference: among plans within 2 % of the fastest the first one
  // wins, so that timing noise does not flip the plan (fewer launches first, then the
  // one-lane-per-site kernel before the split ones; 2D and 3D: the whole y half in one
  // launch before the split one, taller bands first).
  std::vector<qlg_tuning> cand;
  if (c->p.ndim == 1) {
    for (int S = kMaxSteps1D; S >= 1; --S)
      for (int split = 0; split <= 2; ++split)
        if (S <= (split == 0 ? kMaxSteps1D : split == 1 ? kTunePairSteps : kMaxStepsLanes))
          cand.push_back(qlg_tuning{S, 0, c->tuning.use_graph, split});
  } else {
    // powers of two, plus the smallest band heights whose tile count fits k waves per SIMD
    // (k = 1..4): fewer halo rows without a tail of SIMDs that hold one wave more
    std::vector<int> rows = {16, 32, 64, 128};
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
    const int64_t nsimd = 4 * (int64_t)cus;
    auto ntiles = [&](int r) {
      int64_t t = 0;
      for (const auto& d : c->L.inst) { int a, b; tiles_2d(d.nx, d.ny, r, &a, &b); t += (int64_t)a * b * d.nz; }
      return t;
    };
    for (int k = 1; k <= 4 && nsimd > 0; ++k) {
      int r = kMinTileRows;
      while (r < kMaxTileRows && ntiles(r) > k * nsimd) ++r;
      if (ntiles(r) <= k * nsimd && std::find(rows.begin(), rows.end(), r) == rows.end()) rows.push_back(r);
    }
    std::sort(rows.begin(), rows.end(), [](int x, int y) { return x > y; });
    for (int split = 0; split <= 1; ++split)
      for (int r : rows) cand.push_back(qlg_tuning{1, r, c->tuning.use_graph, split});
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(c, QLG_ERR_DEVICE, "event create");
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return fail(c, QLG_ERR_DEVICE, "event create"); }
  std::vector<double> per_step_ms;
  for (const auto& t : cand) {
    c->tuning = t;
    if ((s = build_tiles(c))) break;
    const int S = c->p.ndim == 1 ? t.steps_per_pass : 1;
    // passes read the current copy and write the other one without swapping: the state is
    // unchanged.  The batch of passes is captured once as a hipGraph and replayed, as the runs
    // replay theirs (eager launches would add a dispatch gap per launch, which the plans that
    // split a step into more launches pay more of).  One warm-up replay, then the best of two.
    const int reps = 8;
    hipGraphExec_t exec = nullptr;
    hipError_t e;
    {
      hipStream_t cap = nullptr;
      e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
      hipGraph_t graph = nullptr;
      if (e == hipSuccess) {
        hipStream_t saved = c->stream;
        c->stream = cap;
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        for (int k = 0; k < reps && e == hipSuccess; ++k)
          e = launch_pass(c, S, false, c->copy(c->cur), c->copy(1 - c->cur), nullptr, nullptr, true);
        hipError_t e2 = hipStreamEndCapture(cap, &graph);
        if (e == hipSuccess) e = e2;
        c->stream = saved;
        (void)hipStreamDestroy(cap);
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
    }
    double per_step = 1e300;
    if (e == hipSuccess) e = hipGraphLaunch(exec, c->stream);
    for (int round = 0; round < 2 && e == hipSuccess; ++round) {
      e = hipEventRecord(e0, c->stream);
      if (e == hipSuccess) e = hipGraphLaunch(exec, c->stream);
      if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess) per_step = std::min(per_step, ms / (reps * (double)S));
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (e != hipSuccess) { s = hip_check(c, e, "autotune"); break; }
    per_step_ms.push_back(per_step);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s) return s;
  if (per_step_ms.empty()) return fail(c, QLG_ERR_STATE, "autotune: no candidate plan");
  const double best = *std::min_element(per_step_ms.begin(), per_step_ms.end());
  qlg_tuning best_t = cand[0];
  for (size_t k = 0; k < cand.size(); ++k)
    if (per_step_ms[k] <= 1.02 * best) { best_t = cand[k]; break; }
  c->tuning = best_t;
  c->tuned = true;
  {
    const std::string key = tune_key(c);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best_t;
    tune_file_store(key, best_t);
  }
  return build_tiles(c);
}

qlg_status qlg_set_timing(qlg_ctx* c, int32_t enable) {
  qlg_status s = check_ctx(c);
  if (s) return s;
  c->timing = enable != 0;
  c->time_ms = 0.0;
  c->time_launches = 0;
  return QLG_OK;
}

qlg_status qlg_last_kernel_ms(qlg_ctx* c, double* ms, int64_t* launches) {
  if (!c || !ms || !launches) return QLG_ERR_ARG;
  if (c->broken) return QLG_ERR_STATE;
  *ms = c->time_launches ? c->time_ms / c->time_launches : 0.0;
  *launches = c->time_launches;
  return QLG_OK;
}

}  // extern "C"

namespace qlg {

// Host checks of a parameter block (no device call, no allocation); *msg names the failure.
qlg_status validate_params(const qlg_params* p, const char** msg) {
  if (!p) { *msg = "params is NULL"; return QLG_ERR_ARG; }
  if (p->ndim < 1 || p->ndim > 3) { *msg = "ndim must be 1, 2 or 3"; return QLG_ERR_SHAPE; }
  if (p->dtype != QLG_C64 && p->dtype != QLG_C128) { *msg = "dtype must be QLG_C64 or QLG_C128"; return QLG_ERR_DTYPE; }
  if (p->split != QLG_SPLIT_INTERLEAVED && p->split != QLG_SPLIT_PLAIN) { *msg = "unknown split"; return QLG_ERR_ARG; }
  if (p->nbatch < 1) { *msg = "nbatch must be >= 1"; return QLG_ERR_SHAPE; }
  if (!p->nx) { *msg = "nx is NULL"; return QLG_ERR_ARG; }
  if (p->ndim >= 2 && !p->ny) { *msg = "ny is NULL for a 2D or 3D lattice"; return QLG_ERR_ARG; }
  if (p->ndim == 3 && !p->nz) { *msg = "nz is NULL for a 3D lattice"; return QLG_ERR_ARG; }
  if (!std::isfinite(p->g0) || !std::isfinite(p->g1) || !std::isfinite(p->g2)) { *msg = "couplings must be finite"; return QLG_ERR_ARG; }
  if (!std::isfinite(p->eps) || !(p->eps > 0)) { *msg = "eps must be finite and > 0"; return QLG_ERR_ARG; }
  for (int i = 0; i < p->nbatch; ++i) {
    const int64_t nx = p->nx[i];
    const int64_t ny = p->ndim >= 2 ? p->ny[i] : (p->ny ? p->ny[i] : 1);
    const int64_t nz = p->ndim == 3 ? p->nz[i] : (p->nz ? p->nz[i] : 1);
    if (nx < 1 || ny < 1 || nz < 1 || nx > kMaxExtent || ny > kMaxExtent || nz > kMaxExtent) {
      *msg = "extents must be in [1, 2^30]";
      return QLG_ERR_SHAPE;
    }
    if (p->ndim == 1 && ny != 1) { *msg = "ny must be 1 (or NULL) for ndim == 1"; return QLG_ERR_SHAPE; }
    if (p->ndim < 3 && nz != 1) { *msg = "nz must be 1 (or NULL) for ndim < 3"; return QLG_ERR_SHAPE; }
    if (nx * ny > kMaxSites || nx * ny * nz > kMaxSites) { *msg = "an instance exceeds 2^31-1 sites"; return QLG_ERR_SHAPE; }
  }
  return QLG_OK;
}

// Decoding of nrec observables records of the p->nbatch instances into out[nrec][nbatch];
// false if any is non-finite or, where the record holds a reference norm, drifted beyond the
// dtype's threshold.  No allocation.
bool decode_record_values(const qlg_params& p, const double* rec, int64_t nrec, qlg_obs* out) {
  const int nb = p.nbatch;
  const double meas = std::pow(p.eps, p.ndim);
  const double tol = p.dtype == QLG_C64 ? 1e-4 : 1e-10;
  bool bad = false;
  for (int64_t k = 0; k < nrec * nb; ++k) {
    const double* r = rec + (size_t)k * qlg::kRecord;
    qlg_obs& o = out[k];
    std::memset(&o, 0, sizeof o);
    o.norm_q = meas * r[0];
    o.norm_psi = meas * r[1];
    for (int m = 0; m < 5; ++m) o.pop[m] = meas * r[2 + m];
    o.energy = meas * (r[7] / (p.eps * p.eps) + r[8]);
    o.step = (int64_t)r[qlg::kNObs + 3];
    const int flags = (int)r[qlg::kNObs + 4];
    o.has_overlap = (flags & 1) ? 1 : 0;
    if (o.has_overlap) {
      o.overlap_re = meas * r[qlg::kNObs];
      o.overlap_im = meas * r[qlg::kNObs + 1];
      const double nn = o.norm_psi;
      if (nn > 0) {   // i (nn - ov) / nn
        o.e_overlap_re = o.overlap_im / nn;
        o.e_overlap_im = (nn - o.overlap_re) / nn;
      }
    }
    for (int j = 0; j < qlg::kNObs; ++j) bad |= !std::isfinite(r[j]);
    const double ref = r[qlg::kNObs + 2];
    if ((flags & 2) && ref > 0) {
      const double drift = r[0] / ref - 1.0;
      bad |= !(std::fabs(drift) <= tol);
    }
  }
  return !bad;
}

}  // namespace qlg

// Accessors used by the adjoint implementation (qlg_adjoint.cpp).
namespace qlg {
CtxView ctx_view(qlg_ctx* c) {
  CtxView v;
  v.p = &c->p;
  v.elems_per_copy = c->L.elems_per_copy;
  v.state = c->state;
  v.elem_bytes = c->elem_bytes;
  v.stream = c->stream;
  v.cur = c->cur;
  v.geom = c->geom();
  v.part = c->sc(c->S.obs_part);
  v.res = c->sc(c->S.obs_res);
  v.ext = c->ext;
  return v;
}
hipError_t ctx_aux(qlg_ctx* c, hipStream_t* aux, hipEvent_t** ev) {
  if (!c->aux) {
    // on the context's device, whichever device is current
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != c->device) e = hipSetDevice(c->device);
    if (e != hipSuccess) return e;
    e = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking);
    if (e != hipSuccess) c->aux = nullptr;
    for (auto& x : c->aux_ev) {
      if (e != hipSuccess) break;
      e = hipEventCreateWithFlags(&x, hipEventDisableTiming);
      if (e != hipSuccess) x = nullptr;
    }
    if (e != hipSuccess) {   // leave nothing half made
      for (auto& x : c->aux_ev)
        if (x) (void)hipEventDestroy(x), x = nullptr;
      if (c->aux) (void)hipStreamDestroy(c->aux), c->aux = nullptr;
    }
    const hipError_t r = cur != c->device ? hipSetDevice(cur) : hipSuccess;
    if (e != hipSuccess) return e;
    if (r != hipSuccess) return r;
  }
  *aux = c->aux;
  *ev = c->aux_ev;
  return hipSuccess;
}
qlg_status ctx_fail(qlg_ctx* c, qlg_status s, const char* msg) { return fail(c, s, msg); }
qlg_status ctx_step(qlg_ctx* c, int64_t nsteps) { return qlg_step(c, nsteps); }
bool ctx_broken(const qlg_ctx* c) { return c->broken; }
qlg_status ctx_hip(qlg_ctx* c, hipError_t e, const char* what) { return hip_check(c, e, what); }
}  // namespace qlg
