/* Grouped batches (lupp_batched_solve_grouped): several uniform AoS batches of
 * different sizes in one launch per size class (Section 4.1: size-aware
 * dispatch, with the sizes known to the host). The host lays the groups out
 * as work items (largest sizes first) in the kernel arguments; no device
 * workspace, no grouping kernels, no synchronisation. */
#include <algorithm>
#include <vector>

#include "kernels_ragged.h"
#include "serving.h"

namespace lupp {

/* work items per launch (grid limit: items x 256 threads < 2^32) */
constexpr int64_t kGroupedMaxItems = (int64_t)1 << 23;

int grouped_enqueue(const lupp_group *groups, int ngroups, const uint8_t *lanes, bool factors,
                    hipStream_t st)
{
    return grouped_enqueue_each(groups, nullptr, factors, ngroups, lanes, st);
}

int grouped_enqueue_each(const lupp_group *groups, const uint8_t *factors_of, bool factors,
                         int ngroups, const uint8_t *lanes, hipStream_t st)
{
    std::vector<int> order;
    for (int i = 0; i < ngroups; ++i)
        if (groups[i].batch > 0) order.push_back(i);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return groups[x].n > groups[y].n; });
    for (int cls = 0; cls < kRaggedClasses; ++cls) {
        GroupedArgs a{};
        int64_t items = 0;
        auto flush = [&]() -> hipError_t {
            if (a.ngroups == 0) return hipSuccess;
            const hipError_t e = cls == 0   ? grouped_c0_launch(a, (unsigned)items, st)
                                 : cls == 1 ? grouped_c1_launch(a, (unsigned)items, st)
                                            : grouped_c2_launch(a, (unsigned)items, st);
            a = GroupedArgs{};
            items = 0;
            return e;
        };
        for (int i : order) {
            const lupp_group &g = groups[i];
            if (ragged_class_of(g.n) != cls) continue;
            const int T = lanes[g.n];
            const int64_t per = grouped_per_item(T);
            /* a group larger than one launch's items is split into ranges */
            for (int64_t first = 0; first < g.batch;) {
                if (a.ngroups == kMaxGroups || items == kGroupedMaxItems) {
                    const hipError_t e = flush();
                    if (e != hipSuccess) return hip_err(e);
                }
                const int64_t room = (kGroupedMaxItems - items) * per;
                const int64_t cnt = std::min(g.batch - first, room);
                GroupDesc &d = a.g[a.ngroups++];
                d.A = g.A + first * g.strideA;
                d.b = g.b + first * g.strideB;
                d.ipiv = g.ipiv + first * g.n;
                d.info = g.info + first;
                d.lda = g.lda;
                d.sA = g.strideA;
                d.sB = g.strideB;
                d.batch = cnt;
                d.n = g.n;
                d.lanes = T;
                d.item0 = (int32_t)items;
                d.factors = (factors_of ? factors_of[i] != 0 : factors) ? 1 : 0;
                items += (cnt + per - 1) / per;
                first += cnt;
            }
        }
        const hipError_t e = flush();
        if (e != hipSuccess) return hip_err(e);
    }
    return 0;
}

}  // namespace lupp
