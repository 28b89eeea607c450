// Internal view of a context for the adjoint implementation.
#pragma once

#include "../../include/qlg.h"
#include "qlg_internal.hpp"

namespace qlg {

struct CtxView {
  const qlg_params* p;
  int64_t elems_per_copy;   // complex elements of one padded state copy
  char* state;              // current copy = state + cur * elems_per_copy * elem_bytes
  size_t elem_bytes;
  hipStream_t stream;
  int cur;
  LaunchGeom geom;
  double* part;             // scratch: >= nchunks * 10 doubles
  double* res;              // scratch: >= nbatch * 16 doubles
  ExtPot ext;               // external and chemical potential (constants of the derivative)
};

CtxView ctx_view(qlg_ctx* c);
// The context's second stream (non-blocking, default priority) and four events for ordering
// work between it and the context's stream; made on first use, released by qlg_destroy.
hipError_t ctx_aux(qlg_ctx* c, hipStream_t* aux, hipEvent_t** ev);
qlg_status ctx_fail(qlg_ctx* c, qlg_status s, const char* msg);
qlg_status ctx_step(qlg_ctx* c, int64_t nsteps);
qlg_status ctx_hip(qlg_ctx* c, hipError_t e, const char* what);
bool ctx_broken(const qlg_ctx* c);

}  // namespace qlg
