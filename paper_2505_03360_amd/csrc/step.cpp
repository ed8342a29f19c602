// One time step of the hybrid hot path captured as a HIP graph: regime mask
// (Algorithm 1) and compaction, then the collision operator over exactly the
// cells the mask put in the Boltzmann layer (their count is read on the GPU,
// so a replay needs no host synchronisation and no re-capture when the mask
// changes), scattered into the output rows, then the new regimes copied over
// the old ones for the next step.
#include "bz_internal.hpp"

namespace bz {
void launch_copy_u8(const uint8_t* src, uint8_t* dst, int n, hipStream_t s);
void launch_compact_kinetic(const uint8_t* regime, int ncell, int32_t* idx, int32_t* count, hipStream_t s);
}

struct bz_step {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture = nullptr;
};

extern "C" {

bz_status bz_step_create(const bz_plan* plan, const bz_mask_desc* mask, const bz_step_buffers* b,
                         bz_step** out) {
  bz::clear_error();
  if (!plan || !mask || !b || !out) return bz::fail(BZ_ERR_ARG, "bz_step_create: null argument");
  *out = nullptr;
  if (plan->dim == 2) return bz::fail(BZ_ERR_UNSUPPORTED, "bz_step_create: three velocity dimensions only");
  if (!plan->ws_dev) return bz::fail(BZ_ERR_STATE, "bz_step_create: plan not bound");
  const long ncell = long(mask->nx) * mask->ny;
  if (ncell > plan->capacity)
    return bz::fail(BZ_ERR_NOMEM, "bz_step_create: plan capacity %d < %ld grid cells", plan->capacity, ncell);
  if (!b->f || !b->q || !b->regime_in || !b->regime_out || !b->boltz_idx || !b->counts)
    return bz::fail(BZ_ERR_ARG, "bz_step_create: null buffer");
  if (b->f_dtype != BZ_FP32 && b->f_dtype != BZ_FP64) return bz::fail(BZ_ERR_ARG, "bz_step_create: bad f_dtype");
  if (!plan->project) return bz::fail(BZ_ERR_ARG, "bz_step_create: the step writes FP64 projected output");
  if (b->kinetic_moments && (!b->kin_idx || !b->kin_count || !b->l1dist || !b->rho || !b->ux || !b->uy || !b->T))
    return bz::fail(BZ_ERR_ARG, "bz_step_create: kinetic_moments needs kin_idx, kin_count, l1dist and the fields");
  bz_step* st = new bz_step();
  hipError_t e = hipStreamCreateWithFlags(&st->capture, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete st;
    return bz::fail(BZ_ERR_DEVICE, "bz_step_create: %s", hipGetErrorString(e));
  }
  auto cleanup = [&](bz_status code, const char* what, hipError_t he) {
    if (st->exec) (void)hipGraphExecDestroy(st->exec);
    if (st->graph) (void)hipGraphDestroy(st->graph);
    (void)hipStreamDestroy(st->capture);
    delete st;
    return bz::fail(code, "bz_step_create: %s: %s", what, hipGetErrorString(he));
  };
  e = hipStreamBeginCapture(st->capture, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return cleanup(BZ_ERR_DEVICE, "begin capture", e);
  bz_status rc = BZ_OK;
  if (b->kinetic_moments) {
    // the kinetic cells' fields and L1 distance from their own f
    bz::launch_compact_kinetic(b->regime_in, int(ncell), b->kin_idx, b->kin_count, st->capture);
    bz_moments_out mo{const_cast<double*>(b->rho), const_cast<double*>(b->ux), const_cast<double*>(b->uy), nullptr,
                      const_cast<double*>(b->T), const_cast<double*>(b->l1dist)};
    rc = bz_cell_moments(plan->n, plan->L, b->f, b->f_dtype, b->kin_idx, int(ncell), b->kin_count, &mo, BZ_SCATTER,
                         st->capture);
  }
  if (rc == BZ_OK)
    rc = bz_realizability_mask(mask, b->rho, b->ux, b->uy, b->T, b->eps, b->regime_in, b->l1dist,
                                       b->cell_flags, b->regime_out, b->boltz_idx, b->counts, b->diag,
                                       st->capture);
  if (rc == BZ_OK) {
    bz::Binding bd;
    bd.tables = plan->tables_dev;
    bd.ws = plan->ws_dev;
    bd.capacity = plan->capacity;
    bd.lay = plan->ws;
    rc = bz::launch_collide(plan, bd, b->f, b->f_dtype == BZ_FP32, b->boltz_idx, int(ncell), b->counts, b->q,
                            1, st->capture, false);
  }
  if (rc == BZ_OK) bz::launch_copy_u8(b->regime_out, const_cast<uint8_t*>(b->regime_in), int(ncell), st->capture);
  e = hipStreamEndCapture(st->capture, &st->graph);
  if (rc != BZ_OK) {
    std::string msg = bz_last_error();
    if (st->graph) (void)hipGraphDestroy(st->graph);
    (void)hipStreamDestroy(st->capture);
    delete st;
    return bz::fail(rc, "bz_step_create: capture failed: %s", msg.c_str());
  }
  if (e != hipSuccess) return cleanup(BZ_ERR_DEVICE, "end capture", e);
  e = hipGraphInstantiate(&st->exec, st->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return cleanup(BZ_ERR_DEVICE, "instantiate", e);
  *out = st;
  return BZ_OK;
}

bz_status bz_step_launch(bz_step* st, void* stream) {
  bz::clear_error();
  if (!st) return bz::fail(BZ_ERR_ARG, "bz_step_launch: null step");
  const hipError_t e = hipGraphLaunch(st->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return bz::fail(BZ_ERR_DEVICE, "bz_step_launch: %s", hipGetErrorString(e));
  return BZ_OK;
}

bz_status bz_step_destroy(bz_step* st) {
  bz::clear_error();
  if (!st) return BZ_OK;
  if (st->exec) (void)hipGraphExecDestroy(st->exec);
  if (st->graph) (void)hipGraphDestroy(st->graph);
  if (st->capture) (void)hipStreamDestroy(st->capture);
  delete st;
  return BZ_OK;
}

}  // extern "C"
