// eval_inst_f64.hip -- resident-kernel instantiations for PATH_F64 (one file per path so the
// instantiations compile in parallel).
#include "eval_resident.h"

namespace curob {

const void *const *resident_table_f64() {
  return resident_table<PATH_F64>(std::make_integer_sequence<int, K_COUNT * 4>{});
}

}  // namespace curob
