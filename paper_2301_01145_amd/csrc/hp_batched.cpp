// Batched persistent solve (many independent bounded problems, one launch).
#include "hp_plan.hpp"

namespace hp {

hp_status batched_setup(hp_plan p) {
  return plan_fail(p, HP_E_UNSUPPORTED, "batched plans are not available yet");
}

hp_status batched_solve(hp_plan p) {
  return plan_fail(p, HP_E_UNSUPPORTED, "batched plans are not available yet");
}

}  // namespace hp
