// Tape evaluation kernels for F16 storage (one translation unit per dtype).
#include "fx_tape.hpp"

namespace fx {
FX_TAPE_EVAL_DEFINE(f16_t)
}  // namespace fx
