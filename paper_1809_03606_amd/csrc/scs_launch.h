// Host-side launch description shared between the HIP translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scs_device.h"

namespace polarscs {

struct FsscsLaunch {
  CodeArgs code;  // nodes and crc_tab set
  int D, L, dtype;
  int waves_per_block;
  const void* llr;
  int64_t n_frames;
  uint8_t* payload;
  uint8_t* status;
  scs_stats* stats;
  hipStream_t stream;
};

// Enqueue the fast simplified stack decoder (one frame per wavefront).
hipError_t launch_fsscs(const FsscsLaunch& a);

struct SclLaunch {
  CodeArgs code;  // crc_tab set
  int L, dtype;
  int waves_per_block;
  const void* llr;
  int64_t n_frames;
  uint8_t* payload;
  uint8_t* status;
  scs_stats* stats;
  hipStream_t stream;
};

// LDS bytes of one frame of the list decoder, and the launcher.
size_t scl_lds_bytes(int N, int L);
hipError_t launch_scl(const SclLaunch& a);

}  // namespace polarscs
