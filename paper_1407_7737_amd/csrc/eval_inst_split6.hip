// eval_inst_split6.hip -- resident-kernel instantiations for PATH_SPLIT6 (one file per path so the
// instantiations compile in parallel).
#include "eval_resident.h"

namespace curob {

const void *const *resident_table_split6() {
  return resident_table<PATH_SPLIT6>(std::make_integer_sequence<int, K_COUNT * 4>{});
}

}  // namespace curob
