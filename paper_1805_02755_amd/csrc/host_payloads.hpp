// Host-side payload workers. Each function computes a sub-range of the index
// space with the same FP32 operation sequence per work-item as the GPU
// kernels, so the bits do not depend on which device computed an item.
#pragma once

#include <stdint.h>

#include "../../include/coexec.h"

namespace ce {

struct HostPayloadFns {
  // rows [r0, r1) of the escape-time image; out is the image base
  void (*escape_rows)(const ce_escape_params& p, uint64_t r0, uint64_t r1, uint32_t* out);
  // rows [r0, r1) of the blurred image
  void (*blur5_rows)(const float* in, uint32_t w, uint32_t h, const float* wt, uint64_t r0, uint64_t r1,
                     float* out);
  // bodies [i0, i1)
  void (*nbody_bodies)(const float* pos4, uint32_t n, float eps2, int strict, uint64_t i0, uint64_t i1,
                       float* out4);
  const char* isa;
};

// Picks the widest instruction set the running CPU supports (AVX-512 or
// AVX2+FMA); returns nullptr if the CPU lacks FMA.
const HostPayloadFns* host_payloads();

// N-body integration step of bodies [i0, i1), after the accelerations: on
// entry vel_out4 holds them (as nbody_bodies writes them); on return
// pos_out4 and vel_out4 hold the stepped positions and velocities, with the
// same FP32 operations as the GPU: h = (dt*dt)*0.5, x' = (x + v*dt) + a*h,
// v' = v + a*dt, mass and velocity w copied.
void nbody_step_update(const float* pos4, const float* vel4, float dt, uint64_t i0, uint64_t i1, float* pos_out4,
                       float* vel_out4);

// Binomial option pricing of groups [g0, g1) (four calls per float4 of
// spots), with the GPU's FP32 operations: leaves max(S*f_j - strike, 0), then
// V_j = pu*V_{j+1} + pd*V_j level by level; out4 gets V_0 of each call.
void binomial_groups(const float* spots4, const float* factors, uint32_t steps, float strike, float pu, float pd,
                     uint64_t g0, uint64_t g1, float* out4);

}  // namespace ce
