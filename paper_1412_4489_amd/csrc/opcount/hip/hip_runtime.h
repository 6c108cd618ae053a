// hip/hip_runtime.h for the host operation count (opcount.cpp): the device
// qualifiers are plain host inline functions there.
#pragma once
#define __device__
#define __host__
#define __forceinline__ inline
