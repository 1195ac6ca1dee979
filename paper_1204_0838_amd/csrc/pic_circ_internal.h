// Launchers of the quasi-cylindrical kernels (pic_circ.hip) for the host ABI
// (pic_circ_abi.hip).  Not part of the public C ABI.
#pragma once

#include "pic_circ_device.h"
#include "pic_internal.h"

namespace pic {

size_t circ_tile_lds();
int circ_tile_z();
int circ_tile_r();

hipError_t launch_circ_gather_push(const CircGeom& g, const CircFields& F, const SpeciesDev& s, const PrevDev& prev,
                                   const int* d_count, int max_count, int* err, hipStream_t st);
hipError_t launch_circ_deposit(const CircGeom& g, const SpeciesDev& s, const PrevDev& prev, const int* d_count,
                               int max_count, float q, unsigned long long* acc, hipStream_t st);
// threads: 256, 512 or 1024 per tile workgroup (other values: 512)
hipError_t launch_circ_tile(const CircGeom& g, const CircFields& F, const SpeciesDev& s, const int* toff, int ntz,
                            int ntiles, unsigned long long* acc, int* err, int* rest_n, int* rest_idx, int threads,
                            hipStream_t st);
hipError_t launch_circ_rest(const CircGeom& g, const CircFields& F, const SpeciesDev& s, const int* d_sorted,
                            const int* d_count, const int* rest_n, const int* rest_idx, int max_items,
                            unsigned long long* acc, int* err, hipStream_t st);
hipError_t launch_circ_jfinal(const CircGeom& g, unsigned long long* acc, float* const J[9], int zero,
                              hipStream_t st);
hipError_t launch_circ_bhalf(const CircGeom& g, float* const F[2][3][3], float h, hipStream_t st);
hipError_t launch_circ_efull(const CircGeom& g, float* const F[2][3][3], float* const J[9], hipStream_t st);
hipError_t launch_circ_laser(const CircGeom& g, float* const F[2][3][3], int iz, int which, double coef,
                             double inv_w2, hipStream_t st);
hipError_t launch_circ_clear_plane(const CircGeom& g, float* const F[2][3][3], int iz, hipStream_t st);
hipError_t launch_circ_inject(const CircGeom& g, const SpeciesDev& s, long long shift, int zb, int ze, int r_cells,
                              int ppc, unsigned long long seed, double z_start, double ramp, double n_plateau,
                              double dz, double dr, int* d_count, int capacity, int* err, hipStream_t st);
hipError_t launch_circ_diag(const CircGeom& g, const CircFields& F, float* const Jp[9], const SpeciesDev* s,
                            const int* const* d_count, const double* q, const double* m, const int* max_count,
                            int nspecies, double* out, unsigned long long* cnt, unsigned int* jmax, hipStream_t st);

}  // namespace pic
