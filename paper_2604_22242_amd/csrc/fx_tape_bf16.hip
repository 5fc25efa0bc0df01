// Tape evaluation kernels for BF16 storage (one translation unit per dtype).
#include "fx_tape.hpp"

namespace fx {
FX_TAPE_EVAL_DEFINE(bf16_t)
}  // namespace fx
