// Device scratch and host buffers of the entry point that allocates nothing
// (abdf_solve_noalloc).
#pragma once

#include <cstddef>
#include <string>

#include "engine.hpp"

namespace abdf {

// Bytes of the per-device scratch array.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
// Slots its host buffers hold.
constexpr int kNoAllocMaxSlots = 4096;

// The device address of this device's scratch array (looked up once per
// device, the first time the device asks) and its host buffers.  Calls on one
// device share both.  Returns an abdf_status.
int noalloc_workspace(int device, void **scratch_ptr, HostBuffers *host, std::string &err);

}  // namespace abdf
