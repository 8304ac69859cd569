// Host-side launch helpers shared by the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>

namespace ap {

// Raise the dynamic-LDS limit for launches above 64 KiB (gfx950 has 160 KiB per
// workgroup).  Best effort: a launch that still exceeds the limit fails and is
// reported by the hipGetLastError() that follows it.
template <typename K>
inline void prep_lds(K kernel, size_t bytes) {
  if (bytes > 65536) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              int(bytes));
    (void)hipGetLastError();
  }
}

// switch over the supported grid sizes with NX a constant in CALL
#define AP_DISPATCH_NX(NXV, CALL)                        \
  switch (NXV) {                                         \
    case 64: { constexpr int NX = 64; return CALL; }     \
    case 128: { constexpr int NX = 128; return CALL; }   \
    case 256: { constexpr int NX = 256; return CALL; }   \
    case 512: { constexpr int NX = 512; return CALL; }   \
    case 1024: { constexpr int NX = 1024; return CALL; } \
    case 2048: { constexpr int NX = 2048; return CALL; } \
    default: return hipErrorInvalidValue;                \
  }

#define AP_DISPATCH_NX_INT(NXV, CALL)                    \
  switch (NXV) {                                         \
    case 64: { constexpr int NX = 64; return CALL; }     \
    case 128: { constexpr int NX = 128; return CALL; }   \
    case 256: { constexpr int NX = 256; return CALL; }   \
    case 512: { constexpr int NX = 512; return CALL; }   \
    case 1024: { constexpr int NX = 1024; return CALL; } \
    case 2048: { constexpr int NX = 2048; return CALL; } \
    default: return 0;                                   \
  }

}  // namespace ap
