// Tape evaluation kernels for F64 storage (one translation unit per dtype).
#include "fx_tape.hpp"

namespace fx {
FX_TAPE_EVAL_DEFINE(double)
}  // namespace fx
