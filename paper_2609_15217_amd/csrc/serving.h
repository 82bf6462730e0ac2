/* Internal calls of the serving loop (server.cpp) into the rest of the
 * library: merged launches of several requests and the settings of the
 * caller's context. */
#ifndef LUPP_SERVING_H
#define LUPP_SERVING_H

#include "internal.h"

namespace lupp {

/* grouped_enqueue with a factors choice per group (factors_of[i] != 0: write
 * group i's factors back; NULL: `factors` for every group). */
int grouped_enqueue_each(const lupp_group *groups, const uint8_t *factors_of, bool factors,
                         int ngroups, const uint8_t *lanes, hipStream_t st);

/* The fused Newton update of nsets point sets of one law (same tol, maxit,
 * and all with or all without a tangent) in one launch per 24 sets. */
int constitutive_launch_grouped(const lupp_points *sets, int nsets, const lupp_law *law,
                                double tol, int maxit, hipStream_t stream);

/* Copy the tunable settings (dispatch and ragged tables, forced variant,
 * pivoting rule, Newton mapping) of src into dst. */
void ctx_copy_settings(lupp_ctx *dst, const lupp_ctx *src);
/* Whether lupp_batched_solve on ctx pivots textbook-style with the
 * size-aware dispatch (no tile-local pivoting, no forced variant): then its
 * results are those of the grouped path. */
bool ctx_textbook_dispatch(const lupp_ctx *ctx);
/* The context's lanes per size of the ragged and grouped paths. */
const uint8_t *ctx_ragged_lanes(const lupp_ctx *ctx);

}  // namespace lupp

#endif
