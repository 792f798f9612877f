// Instantiation of the Hogwild and SNAPSHOT-contribution kernels for f32 tables, orders = 3.
#include "sgd_kernels.hpp"

namespace lh {
LH_DEFINE_LAUNCHERS(float, 3)
}  // namespace lh
