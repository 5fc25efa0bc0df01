// Compilation of generated kernel source through the driver at first use
// (Sec. 3: the backend compiles each embedded kernel source once, on the fly,
// and reuses it).  One process-wide cache keyed by the source text holds the
// code object of every compiled source; each device loads its module at its
// first launch.  Used by both source modes: the run-time one (text from a
// tape's node list) and the compile-time one (text from an expression's
// type).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fx {

struct jit_program;  // a compiled source (lives until the process ends)

// Compile `src` (len bytes) for gfx950 with the library's flags (-O3, IEEE
// divide and sqrt, denormals kept, no packed FP32 instructions), or find it in
// the cache.  *compile_ms: milliseconds spent compiling (0 if it was cached).
int jit_obtain(const char* src, size_t len, jit_program** prog, double* compile_ms);

// Kernel `name` of `prog` on the current device, loading its module there at
// first use.
int jit_function(jit_program* prog, const char* name, hipFunction_t* fn);

// Launch with kernelParams-style arguments; refuses grids beyond the limits.
int jit_launch(hipFunction_t f, int64_t gx, int64_t gy, int block, void** args, hipStream_t st);

}  // namespace fx
