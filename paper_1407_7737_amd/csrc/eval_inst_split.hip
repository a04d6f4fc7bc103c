// eval_inst_split.hip -- resident-kernel instantiations for PATH_SPLIT (one file per path so the
// instantiations compile in parallel).
#include "eval_resident.h"

namespace curob {

const void *const *resident_table_split() {
  return resident_table<PATH_SPLIT>(std::make_integer_sequence<int, K_COUNT * 4>{});
}

}  // namespace curob
