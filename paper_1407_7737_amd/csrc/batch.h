// batch.h -- batched populations in one persistent launch replayed as a HIP graph.
#pragma once
