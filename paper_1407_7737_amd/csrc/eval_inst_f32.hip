// eval_inst_f32.hip -- resident-kernel instantiations for PATH_F32 (one file per path so the
// instantiations compile in parallel).
#include "eval_resident.h"

namespace curob {

const void *const *resident_table_f32() {
  return resident_table<PATH_F32>(std::make_integer_sequence<int, K_COUNT * 4>{});
}

}  // namespace curob
