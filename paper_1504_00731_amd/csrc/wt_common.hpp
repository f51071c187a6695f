// Host/device qualifiers.  The arithmetic headers are compiled for gfx950 by
// hipcc and, for the CPU checks of the kernel arithmetic, by a host compiler.
#pragma once

#if defined(__HIPCC__) || defined(__HIP__)
#include <hip/hip_runtime.h>
#define WT_HD __host__ __device__ __forceinline__
#else
#define WT_HD inline
#endif
