// AOS solve of the phi sub-problem (constant A_l), see sr_aos.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "sr_device.hpp"

namespace sr {

constexpr int kAosMaxK = 64;   // largest truncation radius of the inverse circulants
// floats of a context's device tap buffer (filled by aos_tap_buffer)
constexpr int kAosTapFloats = ((2 * (kAosMaxK + 1) + 3) & ~3) + 2 * 208;

// FP64 entries c_0..c_K of the inverse of the periodic (1 - 2 tau mu D) on
// n points, truncated where they fall below 1e-9 c_0, into taps[0..kAosMaxK]
// (zero beyond K).  Returns K, or -1 when the cut needs K > kAosMaxK or more
// offsets than the n points hold.
int aos_taps(int n, double tau, double mu, float* taps);
// The device tap buffer of an M x N grid (host memory, kAosTapFloats):
// both directions' taps and their mirrored tables T[m] = c_|m|; with
// Neumann boundaries (bc = 1) the taps of the 2M- and 2N-point circulants.
// Returns -1 (and *Kx or *Ky < 0) when a direction does not truncate.
int aos_tap_buffer(int M, int N, double tau, double mu, int bc, float* buf, int* Kx, int* Ky);
size_t aos_lds_bytes(int Kx, int Ky);
void configure_aos();
// phi_out = AOS solve of the right-hand side r = rhs (tau (N + D + mu Lap phi_in))
// around phi_in, with the taps of aos_tap_buffer (device copy); ev0 / ev1
// (nullable): events recorded at the kernel's start and end.
// bc: 0 periodic, 1 Neumann (mirrored reads).
void launch_aos(int M, int N, int bc, const float* rhs, const float* phi_in, float* phi_out, const float* taps,
                int Kx, int Ky, float taumu, int nz, DevScal* sc, hipStream_t st, hipEvent_t ev0 = nullptr,
                hipEvent_t ev1 = nullptr);

}  // namespace sr
