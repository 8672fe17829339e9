// Host-side launchers of the HIP kernels (declarations shared by the runtime translation unit).
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_ms_device.hpp"

namespace lbmms {

// compiled launch shapes of a lattice; `compacted` adds the 3D fluid-compacted columns (TY 12, 16)
int tile_options(int lattice, bool compacted, int* ty, int* cz, int cap);
// workgroups of the 3D step (64 x ty columns) resident per CU on the current device, 0 on error
int step3d_resident_blocks(int lattice, int prec, int node_shift, int ty);
// 3D step; ty 12 and 16 select the fluid-compacted columns, which read the per-(column, plane)
// fluid lists coff / cpos (global-shift storage in 32 or 16 bits)
hipError_t launch_step(hipStream_t st, const StepArgs& a, int lattice, int prec, int node_shift,
                       int ty, int cz, int nblocks, const unsigned* coff, const unsigned short* cpos);
// 2D work-list step: insts = instance table of this step's parity, tiles = 2 int4 per tile;
// 32 ty lanes per workgroup, rows = 0 for fixed 64 x ty tiles, else the packed tiles' row limit
hipError_t launch_step2d(hipStream_t st, const StepArgs* insts, const int4* tiles,
                         const unsigned* ent, int ntiles, int lattice, int prec, int node_shift, int ty,
                         int rows);
hipError_t launch_init(hipStream_t st, const StepArgs& a, int lattice, int prec, int ns,
                       const double* X, double u0, double u1);
hipError_t launch_residual(hipStream_t st, const StepArgs& a, int lattice, int prec, int ns,
                           double* snap, int update, double* partial, int nblocks, double* out);
// One instance of a batch in the batched residual check: its window snapshot, its partial sums,
// its flags and whether it is still on the work list.
struct ResidualSlot {
    double* snap;           // X at the window start [2][NF] (updated)
    double* partial;        // per-block partial sums [nblocks][8]
    const unsigned* flags;  // the step's flags (the first 16 bytes are copied out)
    int active;             // 0: the instance left the work list and is skipped
    int pad;
};
// the residual reduction of every active instance in two launches: out[k][0..7] as launch_residual
// writes them for instance k, out[k][8..9] its first 16 flag bytes; tab = the instance table of
// the current parity
hipError_t launch_residual_batch(hipStream_t st, const StepArgs* tab, const ResidualSlot* slots,
                                 int count, int lattice, int prec, int ns, int update, int nblocks,
                                 double* out);
hipError_t launch_faces(hipStream_t st, const StepArgs& a, int lattice, int prec, int ns,
                        double* partial, int nblocks, double* out);
hipError_t launch_fields(hipStream_t st, const StepArgs& a, int lattice, int prec, int ns, double* X);
hipError_t launch_populations(hipStream_t st, const StepArgs& a, int lattice, int prec, int ns,
                              int s, int q, double* out);
hipError_t launch_paper_profile(hipStream_t st, const StepArgs& a, double Qs0, double Qs1,
                                double* prof, double* X);

// Advective coupling (lbm_ms_advect.hip): the velocity model's buffers and constants of one step.
struct AdvArgs {
    const void* gin;    // velocity model, post-collision populations of the previous step [Q][P]
    void* gout;         // ... of this step
    const double* xc;   // X of this step per compact node [2][NF] (written by the first pass)
    const double* uin;  // node velocity of the previous step [3][NF]
    double* uout;       // node velocity of this step [3][NF]
    double Qt;          // total lattice outflow per open outlet node, Q_1 + Q_2
    double om_flow;     // 1 / tau_flow
    double nh0, nh1, nh2, nht;  // -nu_s and their sum: the direction of the electrode fluxes
    double eps2;        // square of the flux regularizer
    const int* vox;     // voxel index of each compact node [NF] (the passes run over fluid nodes)
};
// one coupled step: X pass into xw (= v.xc), then the step; FP64 or FP32 storage, every lattice
hipError_t launch_adv_step(hipStream_t st, const StepArgs& a, const AdvArgs& v, double* xw,
                           int lattice, int prec);
// velocity model at rest into v.gout, zero node velocities in v.uout and u_other
hipError_t launch_adv_rest(hipStream_t st, const StepArgs& a, const AdvArgs& v, double* u_other,
                           int lattice, int prec);
// u_M = (ucur + uprev) / 2 times scale into out[3][N] (solid voxels 0)
hipError_t launch_adv_velocity(hipStream_t st, const StepArgs& a, const double* ucur,
                               const double* uprev, double scale, double* out, int lattice,
                               int prec);

}  // namespace lbmms
