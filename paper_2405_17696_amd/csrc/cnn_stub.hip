#include "cnn.h"
namespace helm {
int cnn_prepare(cnn_net*, const helm_op*, hipStream_t) { return fail(HELM_EINVAL, "CNN module not built"); }
int cnn_apply_masked(cnn_net*, const helm_op*, const void*, const double*, int, void*, int, const RhsState*, int, int,
                     hipStream_t) {
    return fail(HELM_EINVAL, "CNN module not built");
}
void cnn_release_cache(helm_op*) {}
}  // namespace helm
