/* Ragged (mixed-size) batches. */
#include "internal.h"

namespace lupp {

int ragged_launch(lupp_ctx *ctx, int64_t batch, const int32_t *n, const int64_t *offA,
                  const int64_t *offB, double *A, double *b, int32_t *ipiv, int32_t *info,
                  bool factors, hipStream_t stream)
{
    (void)ctx; (void)batch; (void)n; (void)offA; (void)offB; (void)A; (void)b; (void)ipiv;
    (void)info; (void)factors; (void)stream;
    return LUPP_E_UNSUPPORTED;
}

}  // namespace lupp
