// Temporary: multigrid and bead entry points until their kernels land.
#include "ek_context.h"

using namespace ek;

size_t ek::bead_state_bytes(int max_beads) { return 4096 + (size_t)max_beads * 64; }
size_t ek::mg_workspace_bytes(int, int, int) { return 256; }
void ek_ctx::mg_setup() {}
ek_status ek_ctx::mg_solve(const double*, double*, int&, double&, double&) {
  return fail(EK_EINVAL, "multigrid not available");
}
BeadTableView ek_ctx::bead_view() const {
  BeadTableView v;
  v.keys = keys;
  v.vals = vals;
  return v;
}
ek_status ek_ctx::beads_deposit() { return EK_OK; }
template <typename T>
ek_status ek_ctx::beads_advance() { return EK_OK; }
template ek_status ek_ctx::beads_advance<float>();
template ek_status ek_ctx::beads_advance<double>();
ek_status ek_ctx::beads_check() { return EK_OK; }
extern "C" ek_status ek_set_polymer(ek_ctx* ctx, int32_t, const double*, const double*,
                                    const double*, const ek_polymer_params*) {
  return ctx ? ctx->fail(EK_EINVAL, "polymer not available") : EK_EINVAL;
}
extern "C" ek_status ek_get_beads(ek_ctx* ctx, double*, double*) {
  return ctx ? ctx->fail(EK_EINVAL, "polymer not available") : EK_EINVAL;
}
