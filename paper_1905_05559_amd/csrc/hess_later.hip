// Entry points not yet implemented in this build step.
#include "api_internal.h"

namespace hs {
hess_status topk_workspace(hess_ctx* ctx, const hess_mlp*, const hess_data*, int64_t, const hess_eig_opts*,
                           size_t*) {
  return fail(ctx, HESS_E_UNSUPPORTED, "hess_topk_eig not built yet");
}
hess_status predvar_workspace(hess_ctx* ctx, const Model&, int, int64_t, size_t*) {
  return fail(ctx, HESS_E_UNSUPPORTED, "hess_predvar not built yet");
}
}  // namespace hs

extern "C" {
hess_status hess_topk_eig(hess_ctx* ctx, const hess_mlp*, const hess_data*, int64_t, const hess_eig_opts*,
                          double*, double*, hess_eig_info*, void*, size_t) {
  return hs::fail(ctx, HESS_E_UNSUPPORTED, "hess_topk_eig not built yet");
}
hess_status hess_predvar(hess_ctx* ctx, const hess_mlp*, int64_t, const double*, const double*, double, int64_t,
                         const void*, const int32_t*, double*, void*, size_t) {
  return hs::fail(ctx, HESS_E_UNSUPPORTED, "hess_predvar not built yet");
}
}
