// Tape evaluation kernels for F32 storage (one translation unit per dtype).
#include "fx_tape.hpp"

namespace fx {
FX_TAPE_EVAL_DEFINE(float)
}  // namespace fx
