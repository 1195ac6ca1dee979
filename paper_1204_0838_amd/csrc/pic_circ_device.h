// Quasi-cylindrical (m = 0, 1) particle step: device building blocks shared
// by the fused tiled kernel, the split kernels and the rest pass, so that
// all paths agree bit for bit (same FP32 arithmetic, int64 fixed-point
// current summed in any order).
//
// Fields per mode and component on a (z, r) grid, z fastest, FP32: channel
// 0 = m 0, 1 = Re m 1, 2 = Im m 1.  Staggering (z, r): E_z (1/2, 0),
// E_r (0, 1/2), E_th (0, 0), B_z (0, 1/2), B_r (1/2, 0), B_th (1/2, 1/2).
// Modes: F = F_0 + Re(F_1 exp(-i th)).  Particles: Cartesian (x, y) FP32
// absolute, z as cell index + FP32 offset, u FP32, w the macroparticle's
// charge weight (n x volume), cell = iz + nz * ir (storage z).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic_device.h"

namespace pic {

struct CircGeom {
    int nz, nr;
    int ncell;            // nz * nr
    int window;           // 1: z is a moving-window circular buffer
    int origin;           // storage z index of window cell 0
    int kill;             // particles outside window cells [kill, nz - 1 - kill] are removed
    int wall;             // particles at r >= (nr - wall) dr are removed
    float dz, dr, dt;
    float inv_dz, inv_dr;
    float dtdz;           // dt / dz
};

// Component order: 0 z, 1 r, 2 th; field planes F[f][c][ch] with f 0 = E, 1 = B.
struct CircFields {
    const float* F[2][3][3];
};

// Current accumulator channels (int64, 2^-40 fixed point):
// 0..2 J_z flux (m0, Re m1, Im m1), 3..5 J_r flux, 6 J_th m0, 7..8 J_th m1 rate.
constexpr int kCircChannels = 9;

__device__ __forceinline__ int circ_zwin(const CircGeom& g, int iz) {
    if (!g.window) return iz;
    const int w = iz - g.origin;
    return w < 0 ? w + g.nz : w;
}

// Density-conserving radial weight of node K+1 for a particle at (K + s) dr.
__device__ __forceinline__ float circ_fr(int K, float s) {
    return fmaf(s * (1.0f - s), 1.0f / (2.0f * (2.0f * (float)K + 1.0f)), s);
}

// Radial position: cell K and offset s of r; r computed in FP32.
__device__ __forceinline__ void circ_rcell(float x, float y, float inv_dr, float& r, int& K, float& s) {
    r = sqrtf(fmaf(x, x, y * y));
    const float t = r * inv_dr;
    K = (int)floorf(t);
    s = t - (float)K;
}

}  // namespace pic
