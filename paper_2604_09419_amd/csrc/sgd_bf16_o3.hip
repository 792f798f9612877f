// Instantiation of the Hogwild and SNAPSHOT-contribution kernels for bf16 tables, orders = 3.
#include "sgd_kernels.hpp"

namespace lh {
LH_DEFINE_LAUNCHERS(uint16_t, 3)
}  // namespace lh
