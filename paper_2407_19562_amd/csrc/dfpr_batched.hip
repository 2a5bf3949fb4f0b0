// Many graphs' Dynamic Frontier updates.
#include "dfpr_common.h"

namespace dfpr {

int run_rank(dfpr_graph *g, int kind, dfpr_stats *st);

int update_many(dfpr_graph *const *gs, int32_t count, dfpr_stats *stats) {
  int worst = DFPR_OK;
  for (int32_t i = 0; i < count; ++i) {
    const int rc = run_rank(gs[i], 2, stats ? stats + i : nullptr);
    if (rc < 0) return rc;
    if (rc > worst) worst = rc;
  }
  return worst;
}

}  // namespace dfpr
