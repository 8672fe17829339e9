// Host-side launchers of the HIP kernels (declarations shared by the runtime translation unit).
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_ms_device.hpp"

namespace lbmms {

int tile_options(int lattice, int* ty, int* cz, int cap);
// workgroups of the 3D step (64 x ty columns) resident per CU on the current device, 0 on error
int step3d_resident_blocks(int lattice, int prec, int node_shift, int ty);
hipError_t launch_step(hipStream_t st, const StepArgs& a, int lattice, int prec, int node_shift,
                       int ty, int cz, int nblocks);
// 2D work-list step: insts = instance table of this step's parity, tiles = 2 int4 per tile;
// 32 ty lanes per workgroup, rows = 0 for fixed 64 x ty tiles, else the packed tiles' row limit
hipError_t launch_step2d(hipStream_t st, const StepArgs* insts, const int4* tiles,
                         const unsigned* ent, int ntiles, int lattice, int prec, int node_shift, int ty,
                         int rows);
hipError_t launch_init(hipStream_t st, const StepArgs& a, int lattice, int prec, int ns,
                       const double* X, double u0, double u1);
hipError_t launch_residual(hipStream_t st, const StepArgs& a, int lattice, int prec, int ns,
                           double* snap, int update, double* partial, int nblocks, double* out);
hipError_t launch_faces(hipStream_t st, const StepArgs& a, int lattice, int prec, int ns,
                        double* partial, int nblocks, double* out);
hipError_t launch_fields(hipStream_t st, const StepArgs& a, int lattice, int prec, int ns, double* X);
hipError_t launch_populations(hipStream_t st, const StepArgs& a, int lattice, int prec, int ns,
                              int s, int q, double* out);
hipError_t launch_paper_profile(hipStream_t st, const StepArgs& a, double Qs0, double Qs1,
                                double* prof, double* X);

}  // namespace lbmms
