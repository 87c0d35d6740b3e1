// Host-side launchers of the kernels (one translation unit per kernel group).
#pragma once

#include "common.h"

namespace ibm {

// Lanes per membrane node in the batched coupling kernels (spreading and
// interpolation): the 3- and 4-point deltas take four stencil nodes per
// lane, so that the many small membranes of a batch make fewer, fuller
// blocks.  The kernels and the batches' work-item tables both use it.
__host__ __device__ constexpr int batch_group_size(int m) {
  return m == 2 ? 8 : (m == 3 ? 8 : 16);
}

// Events that take the start and end timestamps of one kernel's own dispatch
// (hipExtLaunchKernel), so that their elapsed time is the kernel's execution
// alone, without the launch gaps that marker events around it include.
struct DispatchTimer {
  hipEvent_t start, stop;
};

// lbm_kernels.hip
// variant: tuning bits of the collide-stream kernel (see lbm_kernels.hip)
// z0, z1: update only the nodes with z0 <= z < z1 (streaming out of the range
// is included); the default is the whole lattice
// timer: when given, the (single) kernel of this update records its dispatch
void launch_collide_stream(const LatDev &L, int fp16, int src, int par, bool force,
                           bool linear, int variant, hipStream_t s, int z0 = 0, int z1 = -1,
                           const DispatchTimer *timer = nullptr);
// The row form over the rows of rs; false (nothing launched) where the row
// form does not apply (L.tpr == 0)
bool launch_collide_stream_rows(const LatDev &L, int fp16, int src, int par, bool force,
                                bool linear, const RowSet &rs, hipStream_t s);
void launch_init_equilibrium(const LatDev &L, int fp16, int dst, double uw, hipStream_t s);
void launch_get_field(const LatDev &L, int fp16, int src, int gpar, int what, double *out,
                      hipStream_t s);
void launch_set_pops(const LatDev &L, int fp16, int dst, const double *in, hipStream_t s);
void launch_fill_u32(void *p, long long n, uint32_t v, hipStream_t s);
// FP64 mass and momentum of the populations in buffer src into out[4] (device),
// with totals_parts(L) partial sums in part (device)
int totals_parts(const LatDev &L);
void launch_totals(const LatDev &L, int fp16, int src, double4 *part, double *out, hipStream_t s);
void launch_tangent_collide_stream(const LatDev &L, const TanDev &T, int src, int par, bool linear,
                                   hipStream_t s);
void launch_tangent_init(const LatDev &L, const TanDev &T, int dst, int profile, int linear,
                         hipStream_t s);
void launch_get_tangent_pops(const LatDev &L, const TanDev &T, int src, double *out,
                             hipStream_t s);
void launch_adj_velocity(const LatDev &L, const AdjDev &A, const float *f1, int par, int step,
                         int cur, hipStream_t s);
void launch_adj_collide_stream(const LatDev &L, const AdjDev &A, const float *f0, int par, int step,
                               int cur, bool linear, hipStream_t s);
long long adj_couette_blocks(const LatDev &L);
void launch_adj_couette_start(const LatDev &L, const AdjDev &A, int cur, int linear,
                              double *partial, hipStream_t s);
void launch_batch_collide_stream(const BatchDev &B, int fp16, int src, int par, bool linear,
                                 hipStream_t s, const DispatchTimer *timer = nullptr);

// membrane_kernels.hip
void launch_reference_geometry(const MemDev &M, Ctrl *ctrl, hipStream_t s);
// box: sum overlapping stencils of each block in an LDS box first
void launch_spread(const LatDev &L, const MemDev &M, int par, bool box, hipStream_t s);
// advect: 0 Euler, 1 Adams-Bashforth with the stored velocity of the previous step
// mode: 0 lattice velocities per stencil node from the populations, 1 per
// block in an LDS box, 2 from the node-velocity field (a pass over the
// nodes the step's stencils marked first)
void launch_interp_advect(const LatDev &L, const MemDev &M, int fp16, int fsrc, int par,
                          int advect, int mode, hipStream_t s);
void launch_recenter(const MemDev &M, hipStream_t s);
// Spreading of step (par), and interpolation of the step whose new
// populations are in buffer fsrc, each carrying the force-free lattice update
// of the rows of rs in buffer fsrc (row form)
void launch_spread_far(const LatDev &L, const MemDev &M, int par, bool box, int fp16, bool linear,
                       int fsrc, const RowSet &rs, hipStream_t s);
void launch_interp_far(const LatDev &L, const MemDev &M, int fp16, int fsrc, int par, int advect,
                       int mode, bool linear, const RowSet &rs, hipStream_t s);
// min and max over the membrane nodes of floor(lattice z) and floor(lattice
// y) into ctrl->zmin, zmax, ymin, ymax
void launch_node_range(const MemDev &M, Ctrl *ctrl, hipStream_t s);
// batched coupling kernels: each run's stencil-box mode from its MemDev cmode
void launch_batch_spread(const BatchDev &B, int par, hipStream_t s);
void launch_batch_interp(const BatchDev &B, int fp16, int fsrc, int par, int advect, hipStream_t s);
// The whole batched step (all four phases, every run) as one cooperative
// launch of co-resident blocks with grid barriers between the phases; only
// for batches whose runs all use the row form (L.tpr > 0).  Returns 0, or -1
// if the launch was refused.
int launch_batch_persistent(const BatchDev &B, int fp16, int src, int par, int advect, bool linear,
                            hipStream_t s);
void launch_observables(const MemDev &M, Ctrl *ctrl, hipStream_t s);
// observables of the mesh x + h dx into obs [n_caps][16]
void launch_observables_shifted(const MemDev &M, Ctrl *ctrl, const float4 *dx, double h,
                                double *obs, hipStream_t s);
// dD/dx of capsule c (reverse differentiation of the observables) into the
// capsule's rows of grad (FP32, internal node order; other rows untouched),
// or as FP64 [nn][3] rows in the caller's node order
void launch_obs_grad(const MemDev &M, int c, float4 *grad, hipStream_t s);
void launch_obs_grad64(const MemDev &M, int c, double *grad, hipStream_t s);
void launch_adj_interp(const LatDev &L, const MemDev &M, const AdjDev &A, const float *f1, int par,
                       int step, hipStream_t s);
void launch_adj_spread(const LatDev &L, const MemDev &M, const AdjDev &A, hipStream_t s);
void launch_adj_fem(const LatDev &L, const MemDev &M, const AdjDev &A, hipStream_t s);
void launch_tangent_spread(const LatDev &L, const MemDev &M, const TanDev &T, int par,
                           hipStream_t s);
void launch_tangent_interp(const LatDev &L, const MemDev &M, const TanDev &T, int fsrc, int par,
                           hipStream_t s);
void launch_get_mesh(const MemDev &M, double *xyz, double *F, double *u, hipStream_t s);

}  // namespace ibm
