// Adjoint entry points of include/qlg.h.
#include "qlg_adjoint.hpp"

extern "C" {

qlg_status qlg_adjoint_query(const qlg_params* params, int64_t nsteps, int32_t checkpoint_every,
                             size_t* ckpt_bytes, size_t* work_bytes) {
  (void)params; (void)nsteps; (void)checkpoint_every; (void)ckpt_bytes; (void)work_bytes;
  return QLG_ERR_STATE;
}

qlg_status qlg_forward_record(qlg_ctx* ctx, int64_t nsteps, int32_t checkpoint_every, void* ckpt_dev,
                              size_t ckpt_bytes) {
  (void)nsteps; (void)checkpoint_every; (void)ckpt_dev; (void)ckpt_bytes;
  return qlg::ctx_fail(ctx, QLG_ERR_STATE, "adjoint not available in this build");
}

qlg_status qlg_objective_grad(qlg_ctx* ctx, int32_t kind, const void* target_dev, void* lambda_dev,
                              double* value_host, double* dg_host) {
  (void)kind; (void)target_dev; (void)lambda_dev; (void)value_host; (void)dg_host;
  return qlg::ctx_fail(ctx, QLG_ERR_STATE, "adjoint not available in this build");
}

qlg_status qlg_adjoint_step(qlg_ctx* ctx, int64_t nsteps, int32_t checkpoint_every, const void* ckpt_dev,
                            void* lambda_dev, void* work_dev, size_t work_bytes, double* dg_host) {
  (void)nsteps; (void)checkpoint_every; (void)ckpt_dev; (void)lambda_dev; (void)work_dev; (void)work_bytes;
  (void)dg_host;
  return qlg::ctx_fail(ctx, QLG_ERR_STATE, "adjoint not available in this build");
}

}  // extern "C"
