// Scratch of the allocation-free fine-batch entry point (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace ap {

// Bytes of the per-device scratch array: the fine coefficient tables of one
// step size (FP64 and FP32, [8][3][KP] each) and the modal input and output
// states of the batch ([batch][3][KP] complex FP64 each), each part aligned
// to 256 bytes.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;

// Device address of this device's scratch array.  The first call for a device
// must come with that device current; it looks the address up
// (hipGetSymbolAddress) and keeps it.  hipErrorInvalidDevice if `device` is
// not the current device at that first call.
hipError_t noalloc_scratch(int device, void** ptr);

}  // namespace ap
