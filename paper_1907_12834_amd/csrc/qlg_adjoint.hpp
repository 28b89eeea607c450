// Internal view of a context for the adjoint implementation.
#pragma once

#include "../../include/qlg.h"
#include "qlg_internal.hpp"

namespace qlg {

struct CtxView {
  const qlg_params* p;
  const InstDesc* L_inst;
  int64_t elems_per_copy;
  char* state;
  size_t elem_bytes;
  hipStream_t stream;
  int* cur;
  LaunchGeom geom;
};

CtxView ctx_view(qlg_ctx* c);
qlg_status ctx_fail(qlg_ctx* c, qlg_status s, const char* msg);
qlg_status ctx_step(qlg_ctx* c, int64_t nsteps);
bool ctx_broken(const qlg_ctx* c);

}  // namespace qlg
