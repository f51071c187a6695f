// Host/device qualifiers.  The arithmetic headers are compiled for gfx950 by
// hipcc and, for the CPU checks of the kernel arithmetic, by a host compiler.
#pragma once

#if defined(__HIPCC__) || defined(__HIP__)
#include <hip/hip_runtime.h>
#define WT_HD __host__ __device__ __forceinline__
#else
#define WT_HD inline
#endif

// Compiler-only memory barrier in device code: values read from memory (LDS)
// before it are read again after it instead of being held in registers across
// it.  Used at the top of rolled loops whose bodies read the same LDS stencil,
// so the stencil is not hoisted into registers for the whole loop.
#if defined(__HIP_DEVICE_COMPILE__)
#define WT_RELOAD() asm volatile("" ::: "memory")
#else
#define WT_RELOAD() ((void)0)
#endif
