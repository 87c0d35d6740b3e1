/*
 * ibm_lbm.h -- C ABI of the MI355X (gfx950) library for the coupled immersed
 * boundary / lattice Boltzmann / finite element capsule timestep of Krueger,
 * Varnik and Raabe, arXiv:1004.2416.
 *
 * One timestep (Sec. II.C, sub-steps 1-5) is:
 *   1. Skalak membrane forces of every node from its faces (Sec. II.B),
 *   2. spreading of those forces to the lattice through the m-point discrete
 *      delta function (Sec. II.C, Eq. forcespreading),
 *   3. D3Q19 BGK collision with Guo forcing and streaming, periodic in x and
 *      y, moving-wall bounce-back at the z walls (Sec. II.A),
 *   4. interpolation of the new lattice velocity to the old node positions
 *      (Sec. II.C, Eq. velocityinterpolation),
 *   5. Euler advection of the nodes (Sec. II.C, Eq. positionupdate).
 *
 * Units are lattice units (Delta x = Delta t = 1, rho_0 = 1).  The lattice
 * has nx * ny * nz fluid nodes at integer coordinates; walls lie at
 * z = -1/2 (moving with -u_w along x) and z = nz - 1/2 (moving with +u_w).
 *
 * Memory: the library allocates no device memory.  The caller allocates the
 * lattice state and the membrane state as device buffers of the sizes the
 * *_bytes queries report (for instance as torch tensors) and keeps them alive
 * until ibm_destroy; the library never frees them.  Host arrays passed to the
 * library are copied before the call returns.
 *
 * Streams: all work is enqueued on the hipStream_t given at creation.
 * ibm_step and ibm_set_* return without waiting; ibm_get_*, ibm_observables
 * and ibm_synchronize wait for the stream and report device-side errors.
 *
 * Errors: every call returns IBM_OK (0) or a negative IBM_ERR_* code and then
 * ibm_last_error() describes the failure (thread-local string).  No C++
 * exception crosses this interface.  A handle whose device state reported an
 * error stays usable; the flags are cleared when reported.
 *
 * Threading: a handle must not be used from two threads at once.
 */
#ifndef IBM_LBM_H
#define IBM_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------- */
#define IBM_OK 0
#define IBM_ERR_INVALID_ARG (-1)        /* bad size, pointer or parameter       */
#define IBM_ERR_BAD_STATE (-2)          /* call not valid in the handle's state */
#define IBM_ERR_HIP (-3)                /* a HIP runtime call failed            */
#define IBM_ERR_STENCIL_HITS_WALL (-4)  /* a delta stencil reached z < 0 or z >= nz */
#define IBM_ERR_NONFINITE (-5)          /* NaN or Inf found in observables      */
#define IBM_ERR_INVERTED_FACE (-6)      /* a membrane face degenerated or flipped */
#define IBM_ERR_OUTSIDE_SLAB (-7)       /* IBM_OPT_OVERLAP: a stencil reached the
                                           part of the lattice updated without
                                           force; the steps since the last
                                           check are not valid (the slab is
                                           measured again before the next
                                           step)                                */

/* ---- population storage ------------------------------------------------- */
/* Populations are stored as deviations f_i - w_i from the lattice weights in
 * groups of x rows (x fastest), arithmetic in FP32; ibm_get_fields and
 * ibm_set_fields exchange them as [19][nz][ny][nx] FP64 values. */
#define IBM_STORAGE_FP32 0
#define IBM_STORAGE_FP16 1   /* deviations scaled per direction, FP16 storage */
#define IBM_STORAGE_ONE_BUFFER 4 /* or-ed with either: one population buffer
                                    instead of two; the lattice then streams
                                    with the AA pattern only
                                    (IBM_OPT_STREAMING 1, fixed), needs nx a
                                    multiple of 4 and at most 256, and takes
                                    no tangent, adjoint or batch.  Lattices
                                    about 1.6x larger fit the same memory */

/* ---- equilibrium --------------------------------------------------------- */
#define IBM_EQ_QUADRATIC 0   /* Sec. II.A, Eq. (equilibrium)                  */
#define IBM_EQ_LINEAR 1      /* Sec. IV.A linearised form w_i rho (1 + 3 c.u) */

/* ---- field selectors for ibm_get_fields / ibm_set_fields ----------------- */
#define IBM_FIELD_POPS 0   /* [19][nz][ny][nx] f_i(x, t), unshifted, post-streaming */
#define IBM_FIELD_RHO 1    /* [nz][ny][nx] density, Eq. (lbmmomenta0)              */
#define IBM_FIELD_U 2      /* [3][nz][ny][nx] (sum_i c_i f_i + f/2)/rho with the force
                              density f of the last step (zero before the first) */
#define IBM_FIELD_FORCE 3  /* [3][nz][ny][nx] force density f(X) spread in the last step */

/* ---- per-capsule observables (ibm_observables), Sec. III ------------------ */
#define IBM_OBS_V 0        /* enclosed volume                                   */
#define IBM_OBS_CX 1       /* volume centroid x, y, z (unwrapped coordinates)   */
#define IBM_OBS_CY 2
#define IBM_OBS_CZ 3
#define IBM_OBS_D 4        /* Taylor deformation (r_a - r_c)/(r_a + r_c)        */
#define IBM_OBS_THETA 5    /* inclination of the major axis in the xz plane, rad,
                              in (-pi/2, pi/2]; NaN when the two smallest
                              eigenvalues are degenerate                        */
#define IBM_OBS_RA 6       /* semiaxes of the equivalent ellipsoid              */
#define IBM_OBS_RB 7
#define IBM_OBS_RC 8
#define IBM_OBS_AREA 9     /* total face area                                   */
#define IBM_OBS_IXX 10     /* inertia tensor per unit mass about the centroid:
                              xx, yy, zz, xy, xz, yz                           */
#define IBM_OBS_N 16

/* ---- kernel phases (ibm_profile_step) ------------------------------------ */
#define IBM_PHASE_FORCES 0   /* Skalak nodal forces (step 1): formed
                                inside the spreading kernel, so this
                                phase is always empty (0)            */
#define IBM_PHASE_SPREAD 1   /* nodal forces + spreading  (steps 1, 2) */
#define IBM_PHASE_LBM 2      /* collide + stream + walls       (step 3) */
#define IBM_PHASE_INTERP 3   /* interpolation + advection      (steps 4, 5) */
#define IBM_N_PHASES 4

/* ---- options (ibm_set_option) --------------------------------------------- */
#define IBM_OPT_GRAPH 0        /* 1 (default): replay the step chain as a
                                  captured hipGraph; 0: plain launches      */
#define IBM_OPT_EQUILIBRIUM 1  /* IBM_EQ_QUADRATIC (default) or IBM_EQ_LINEAR */
#define IBM_OPT_ADVECTION 2    /* 0 (default): Euler, Eq. (positionupdate);
                                  1: Adams-Bashforth, Sec. II.C             */
#define IBM_OPT_RECENTER 3     /* steps between re-centring of the capsule
                                  frames (default 64, >= 1)                 */
#define IBM_OPT_LBM_VARIANT 4  /* launch variant of the collide-stream kernel,
                                  0..511 (bit 4: four nodes per thread with
                                  whole x rows per wavefront, used when
                                  nx <= 256; else the per-node kernel with
                                  bit 0: two nodes per thread, bit 1:
                                  non-temporal accesses, bit 2: 128-thread
                                  blocks; bits 3 and 5 are ignored;
                                  bit 6, bit 7: the four-node row form in
                                  128- or 64-thread blocks instead of 256;
                                  bit 8: the four-node row form stores the
                                  new populations with ordinary (cached)
                                  writes instead of non-temporal ones;
                                  default 23, plus 256 where one population
                                  buffer takes 48 to 192 MiB, so that most of
                                  it stays in the last-level cache until the
                                  next step reads it);
                                  results are identical, only the speed
                                  differs                                    */
#define IBM_OPT_STENCIL_BOX 6  /* 0..7.  bit 0: spreading, bit 1:
                                  interpolation of the per-node kernels go
                                  through an LDS box spanning the stencils
                                  of each block's nodes (overlapping
                                  stencils are summed, or their lattice
                                  velocities evaluated, once per lattice
                                  node); bit 2 (over bit 1): interpolation
                                  reads the lattice velocity from a field
                                  that one pass evaluates, once per lattice
                                  node, at every node the step's stencils
                                  touch with a nonzero weight.
                                  Default, set when the membrane is
                                  attached unless chosen before: when the
                                  membrane makes at least 256 blocks of
                                  work, 5 (box spreading, the velocity
                                  field) if its stencils cover at least an
                                  eighth of the lattice nodes, else 3 (box
                                  spreading and box interpolation); else 0.
                                  Results agree to FP32 rounding (see also
                                  ibm_autotune)                             */
#define IBM_OPT_OVERLAP 7      /* 1, 2: split the lattice update of
                                  graph-replayed steps at the slab of z
                                  that stencils can reach (the membranes' z
                                  extent plus a margin of 4 + ceil(2 |u_w|
                                  IBM_OPT_RECENTER) lu, rounded out to 4):
                                  the rows outside need no force and run
                                  inside the launches of the spreading
                                  (above the slab) and of the previous
                                  step's interpolation (below), overlapping
                                  them.  The slab is measured again at
                                  every re-centring.  A stencil outside it
                                  makes the next synchronising call fail
                                  with IBM_ERR_OUTSIDE_SLAB.  Used only
                                  without a tangent, with the
                                  row form (nx <= 256), and when the slab
                                  holds at most three quarters of the rows
                                  (value 2), and with value 1 only when at
                                  least 2^20 nodes lie outside it (the
                                  split pays there).  0 (default): off.
                                  Results are those of the plain step       */

#define IBM_OPT_STREAMING 8    /* 0 (default): two population buffers,
                                  collide and push to the neighbours of
                                  the other buffer; 1: the AA pattern in
                                  one buffer: even steps collide in place
                                  into the opposite slots, odd steps gather
                                  from the neighbours and push back (Bailey
                                  et al.'s access pattern): the same 152
                                  bytes per node and step in one
                                  population array, so a lattice created
                                  with IBM_STORAGE_ONE_BUFFER needs only
                                  that one (it streams this way only).
                                  Slower than two buffers on the lattices
                                  measured: the odd step gathers from and
                                  pushes to nine rows per row.  AA
                                  needs the row form (nx <= 256), nx a
                                  multiple of 4 and no tangent; the adjoint
                                  and batches need two buffers.  Changes
                                  only after an even number of steps;
                                  populations can be set then only.  After
                                  an even step the interpolation goes
                                  through the velocity field (stencil-box
                                  bit 2), the one form that reads the
                                  swapped state.
                                  Results are those of two buffers (to FP32
                                  rounding)                                 */
#define IBM_OPT_FP16_MASS 9    /* FP16 storage: 0 (default): every
                                  post-collision value is rounded to FP16
                                  on its own (one step changes a population
                                  by at most 2^-11 of its deviation, and
                                  the roundings move the total mass, by up
                                  to 2^-11 sum_i |f_i - w_i| per node and
                                  step); 1: the rest population, which
                                  stays at its node, also takes back the
                                  mass the node's 18 other stored values
                                  lose to rounding, so the stored values
                                  carry the FP32 mass up to the rounding of
                                  the rest population (Sec. II.A, Eq.
                                  lbmmomenta0: the collision conserves
                                  mass).  Needs the row form (nx <= 256);
                                  the other populations are unchanged     */
#define IBM_STREAM_TWO_BUFFERS 0
#define IBM_STREAM_AA 1

typedef struct ibm_lattice ibm_lattice;

/* Bytes of device memory the lattice state needs (two population buffers,
 * or one with IBM_STORAGE_ONE_BUFFER, two force densities and their tile
 * stamps, the node stamps, the interpolation velocity field, control words).
 * storage: IBM_STORAGE_FP32 or IBM_STORAGE_FP16, optionally or-ed with
 * IBM_STORAGE_ONE_BUFFER. */
int ibm_lattice_bytes(int nx, int ny, int nz, int storage, size_t *bytes);

/* Create a lattice of nx * ny * nz nodes with BGK relaxation time tau > 1/2
 * (Sec. II.A, Eq. lbequation; nu = (tau - 1/2)/3).  dev_state: device buffer
 * of at least ibm_lattice_bytes bytes, 256-byte aligned, owned by the caller.
 * stream: the hipStream_t all work goes to (NULL: the null stream).  The
 * fluid starts at rest (f_i = w_i) with the walls at rest.  On success *out
 * receives the handle. */
int ibm_lattice_create(int nx, int ny, int nz, double tau, int storage,
                       void *dev_state, size_t bytes, void *stream,
                       ibm_lattice **out);

/* Set the wall speed u_w (|u_w| < 0.3): the top wall moves with +u_w along
 * x and the bottom wall with -u_w, shear rate 2 u_w / nz (Sec. II.A).  With
 * init_profile = 1 the populations are also reset to the equilibrium of
 * rho = 1 and the linear profile u_x(z) = u_w (2 z + 1 - nz) / nz, and the
 * step counter to 0. */
int ibm_set_shear(ibm_lattice *lat, double u_w, int init_profile);

/* Bytes of device memory for a membrane of n_caps capsules with the given
 * node and face counts. */
int ibm_membrane_bytes(int n_caps, const int *nodes_per_cap,
                       const int *faces_per_cap, size_t *bytes);

/* Attach the capsules (at most one call per lattice).
 *   xyz  host [sum nodes][3] FP64: stress-free reference shape in lattice
 *        coordinates, which is also the initial shape (Sec. II.B, "all faces
 *        undeformed" at t = 0).  Each capsule keeps an integer origin
 *        floor(mean of its nodes) and FP32 node coordinates relative to it;
 *        the reference geometry is computed in FP64 from those FP32 values.
 *   tri  host [sum faces][3] node indices local to each capsule, counter-
 *        clockwise seen from outside.
 *   ks, ka  host [n_caps] surface shear and area dilation moduli of Skalak's
 *        law (Sec. II.B, Eq. constitutivelaw); C = ka / ks.
 *   m    delta width 2, 3 or 4 (Sec. II.C, Eqs. 2point, 3point, 4point).
 *   dev_mem  device buffer of ibm_membrane_bytes bytes, owned by the caller.
 * nx and ny must be at least m.  Fails with IBM_ERR_STENCIL_HITS_WALL if a
 * stencil would reach a wall and with IBM_ERR_INVERTED_FACE for a degenerate
 * face. */
int ibm_membrane_create(ibm_lattice *lat, int n_caps, const int *nodes_per_cap,
                        const int *faces_per_cap, const double *xyz,
                        const int32_t *tri, const double *ks, const double *ka,
                        int m, void *dev_mem, size_t bytes);

/* Enqueue n >= 0 full timesteps (Sec. II.C sub-steps 1-5; without a membrane,
 * only the lattice update). */
int ibm_step(ibm_lattice *lat, int64_t n);

/* Number of timesteps taken since creation or the last profile reset. */
int64_t ibm_step_count(const ibm_lattice *lat);

/* Write a field (IBM_FIELD_*) as FP64 into the device buffer dst (layouts
 * above), then wait for the stream. */
int ibm_get_fields(ibm_lattice *lat, int what, double *dst_dev);

/* Overwrite the populations (what = IBM_FIELD_POPS) from the device FP64
 * buffer src [19][nz][ny][nx] of unshifted post-streaming values; they are
 * rounded to the storage format.  With the AA pattern (IBM_OPT_STREAMING 1 or
 * a one-buffer lattice) only after an even number of steps, else
 * IBM_ERR_BAD_STATE.  Enqueued, does not wait. */
int ibm_set_fields(ibm_lattice *lat, int what, const double *src_dev);

/* Write node positions (unwrapped lattice coordinates), the nodal forces
 * F_i(t) and the node velocities u_i(t + 1) of the last step as FP64 [nn][3]
 * into device buffers (any may be NULL), nodes in creation order; waits. */
int ibm_get_mesh(ibm_lattice *lat, double *xyz_dev, double *force_dev,
                 double *vel_dev);

/* Overwrite all node positions from host FP64 [nn][3]; each capsule's origin
 * becomes floor(mean of its new nodes).  The reference shape is unchanged.
 * Fails with IBM_ERR_STENCIL_HITS_WALL if a stencil would reach a wall. */
int ibm_set_mesh(ibm_lattice *lat, const double *xyz_host);

/* Shape observables of every capsule (Sec. III): out_host [n_caps][IBM_OBS_N]
 * FP64, from FP64 reductions on the device; waits. */
int ibm_observables(ibm_lattice *lat, double *out_host);

/* Gradient of the Taylor deformation D of one capsule (Sec. III: D from the
 * semiaxes of the ellipsoid with the capsule's inertia tensor) with respect
 * to its node positions, at the current positions, by reverse
 * differentiation of the FP64 observables (eigenvalue derivatives
 * dE_k = v_k^T dI v_k; the eigenvalues must be distinct, which fails for a
 * sphere).  Writes dD/dx as FP64 [nn][3] rows (caller's node order) of the
 * capsule's nodes into the device buffer grad_dev; rows of other capsules are
 * left untouched.  Waits. */
int ibm_deformation_gradient(ibm_lattice *lat, int capsule, double *grad_dev);

/* FP64 totals of the current populations over the whole lattice
 * (Sec. II.A, Eqs. lbmmomenta0/1 summed over all nodes):
 *   out_dev[0] = sum_X sum_i f_i(X)          (mass)
 *   out_dev[1..3] = sum_X sum_i c_i f_i(X)   (momentum of the populations,
 *                                              without the half-force term)
 * The stored FP32 (or FP16) values are converted exactly and summed in FP64
 * in a fixed order, so the same state gives the same bits.  out_dev is a
 * caller device buffer of 4 doubles (8-byte aligned); work_dev a caller
 * device buffer of at least ibm_totals_bytes bytes (32-byte aligned) for the
 * partial sums, free again when the stream has run the call.  Enqueued on the
 * lattice's stream; does not wait.  Errors: IBM_ERR_INVALID_ARG for NULL,
 * misaligned or too small buffers. */
int ibm_totals_bytes(const ibm_lattice *lat, size_t *bytes);
int ibm_lattice_totals(ibm_lattice *lat, void *work_dev, size_t work_bytes, double *out_dev);

/* ibm_lattice_totals without a workspace, for callers that cannot allocate
 * device memory (code under stream capture, serving loops, harnesses that
 * forbid allocation): the same kernels and the same result bits, with the
 * partial sums in a fixed scratch array that the library holds on every GPU
 * it runs on (256 KiB per GPU, kept until the process ends).  Allocates
 * nothing.  Lattices of up to 8192 * 4096 = 33,554,432 nodes; larger ones
 * get IBM_ERR_INVALID_ARG (use ibm_lattice_totals).  All calls on one GPU
 * share its scratch array: calls that may run at the same time on one GPU
 * (different streams, different threads) race and must be serialised by the
 * caller; calls on one stream are ordered by it.  out_dev: caller device
 * buffer of 4 doubles, as for ibm_lattice_totals.  Enqueued; does not wait. */
int ibm_lattice_totals_noalloc(ibm_lattice *lat, double *out_dev);

/* Wait for the stream; report device-side error flags. */
int ibm_synchronize(ibm_lattice *lat);

/* Set an option IBM_OPT_* (see above). */
int ibm_set_option(ibm_lattice *lat, int option, int value);

/* The force box of the split lattice update (IBM_OPT_OVERLAP) that the next
 * graph-replayed steps use: box[0..3] = zlo, zhi, ylo, yhi, the rows
 * zlo <= z < zhi, ylo <= y < yhi (y spans the lattice: ylo = 0, yhi = ny);
 * the whole lattice (0, nz, 0, ny) when the update is not split.  Measures
 * the membranes' extent first if it is stale (waits). */
int ibm_split_box(ibm_lattice *lat, int *box);

/* Choose the fastest collide-stream form (IBM_OPT_LBM_VARIANT) and, with
 * capsules, stencil-box mode (IBM_OPT_STENCIL_BOX) and IBM_OPT_OVERLAP (on
 * only where it splits the update and is faster; query it with
 * ibm_split_box) by timing whole steps of this lattice with HIP events: after 4 x steps_per_trial settling steps,
 * each candidate runs 16 steps and is then timed twice over steps_per_trial
 * steps (rounded up to a multiple of 16), keeping the better time.  The run
 * advances by all these steps (the candidates compute the same update, to
 * FP32 rounding).  chosen (nullable) receives {variant, box mode}.  Waits. */
int ibm_autotune(ibm_lattice *lat, int steps_per_trial, int *chosen);

/* Run n timesteps with plain launches and HIP events between the kernels of
 * every step; ms_per_phase[IBM_N_PHASES] receives the mean duration of each
 * phase per step in milliseconds (a phase that did not run gets 0).  For
 * measurement; waits. */
int ibm_profile_step(ibm_lattice *lat, int64_t n, double *ms_per_phase);

/* Run n timesteps as ibm_profile_step does (plain launches, the whole-lattice
 * update of step 3, Sec. II.A) and store in *ms the mean execution time of
 * the collide-stream kernel alone, in milliseconds: the difference of the
 * start and end timestamps of its own dispatch (hipExtLaunchKernel events),
 * which is what a kernel tracer reports for it; the IBM_PHASE_LBM phase of
 * ibm_profile_step also holds the launch gaps before and after it.  For
 * measurement; waits. */
int ibm_profile_lattice_kernel(ibm_lattice *lat, int64_t n, double *ms);

/* Release the handle (not the caller's device buffers); waits first. */
int ibm_destroy(ibm_lattice *lat);

/* ---- forward sensitivities (tangent-linear model of the timestep) ----------
 * The derivative of the whole state along one parameter direction, advanced
 * beside the timestep by hand-differentiated kernels: the tangent of the
 * Skalak forces (Sec. II.B), of spreading and interpolation including the
 * motion of the delta stencils (Sec. II.C), and of collide + stream +
 * bounce-back (Sec. II.A).  The direction is given by the rates of the
 * parameters: d k_s and d k_alpha per capsule and d u_w; for the reduced
 * shear rate G of Sec. III at fixed C, say, dks = -k_s / G, dka = C dks.
 * Needs FP32 storage and Euler advection. */

/* Device bytes of the tangent state of this lattice (and its membrane). */
int ibm_tangent_bytes(ibm_lattice *lat, size_t *bytes);

/* Attach a tangent state in dev_mem (caller-owned, 256-byte aligned, at least
 * ibm_tangent_bytes) and start it: node and force tangents zero; population
 * tangents zero, or with init_profile = 1 the derivative of the linear
 * Couette start of ibm_set_shear(init_profile = 1) along duw.  dks, dka:
 * host arrays of n_caps rates (NULL without a membrane).  From now on every
 * ibm_step also advances the tangent.  The membrane must be attached first. */
int ibm_tangent_attach(ibm_lattice *lat, const double *dks, const double *dka, double duw,
                       int init_profile, void *dev_mem, size_t bytes);

/* Stop advancing the tangent (dev_mem may then be reused). */
int ibm_tangent_detach(ibm_lattice *lat);

/* Tangent populations, dst_dev [19][nz][ny][nx] FP64 device; waits. */
int ibm_tangent_get_pops(ibm_lattice *lat, double *dst_dev);

/* Tangent node positions and velocities of the last step, [n_nodes][3] FP64
 * device arrays in the caller's node order (either may be NULL); waits. */
int ibm_tangent_get_mesh(ibm_lattice *lat, double *dxyz_dev, double *du_dev);

/* Derivative of every observable (Sec. III) along the tangent: the FP64
 * central difference (obs(x + h dx) - obs(x - h dx)) / (2 h) of the shape
 * observables along the tangent node positions, out_host [n_caps][IBM_OBS_N].
 * h (> 0, in units of the parameter) sets the difference step; waits. */
int ibm_tangent_observables(ibm_lattice *lat, double h, double *out_host);

/* ---- reverse-mode gradient (discrete adjoint of the timestep) --------------
 * The gradient of the Taylor deformation D(T) of one capsule (Sec. III) with
 * respect to every capsule's k_s and k_alpha and the wall speed u_w, by the
 * adjoint of the whole FP32 step: each step reversed (interpolation and
 * advection, the lattice velocity, streaming with the moving-wall
 * bounce-back, BGK + Guo, spreading, the Skalak forces through their Hessian
 * product) with the states recomputed from checkpoints taken every
 * checkpoint_every steps.  D(T)'s own gradient with respect to the node
 * positions is taken by FP64 central differences of the observables.  Needs
 * FP32 storage, Euler advection and no attached tangent. */

/* Device bytes for ibm_adjoint_gradient over `steps` steps. */
int ibm_adjoint_bytes(ibm_lattice *lat, int64_t steps, int checkpoint_every, size_t *bytes);

/* Run `steps` steps from the current state (re-centring off meanwhile) and
 * return D(T) of `capsule` and its gradient: dD_dks, dD_dka host arrays of
 * n_caps values, *dD_duw (with couette_start = 1 including the dependence of
 * a linear Couette start, as set by ibm_set_shear(init_profile = 1), on u_w).
 * dev_mem: caller-owned scratch of ibm_adjoint_bytes bytes, 256-byte aligned.
 * The lattice ends at step T as after ibm_step(steps); after an error its
 * state is unspecified (its options are kept).  Waits. */
int ibm_adjoint_gradient(ibm_lattice *lat, int64_t steps, int checkpoint_every, int capsule,
                         int couette_start, void *dev_mem, size_t bytes, double *D_out,
                         double *dD_dks, double *dD_dka, double *dD_duw);

/* ---- batches of independent runs (Sec. IV parameter studies) ---------------
 * A batch advances many lattices (each with or without capsules, of any size,
 * tau, wall speed and delta width) together: every kernel of the timestep is
 * launched once for all runs, and whole-step sequences are replayed as one
 * captured graph, so many small runs cost a few launches per step instead of
 * a few per run.  The runs stay the caller's handles: fields, meshes and
 * observables are read from them as usual, and they may be stepped alone
 * between batch steps. */
typedef struct ibm_batch ibm_batch;

/* Device bytes the batch of runs[0 .. n_runs-1] needs for its tables. */
int ibm_batch_bytes(int n_runs, ibm_lattice *const *runs, size_t *bytes);

/* Group the runs.  They must share one stream (the batch enqueues on it) and,
 * at every ibm_batch_step, have made the same number of steps and use the same
 * storage, equilibrium and advection options.  dev_mem: caller-owned device
 * buffer of at least ibm_batch_bytes bytes, 256-byte aligned, kept until
 * ibm_batch_destroy.  The runs must outlive the batch; a run may not gain
 * more membrane nodes or faces than it had here (IBM_ERR_BAD_STATE). */
int ibm_batch_create(int n_runs, ibm_lattice *const *runs, void *dev_mem, size_t bytes,
                     ibm_batch **out);

/* Enqueue n timesteps of every run (Sec. II.C, sub-steps 1-5); asynchronous.
 * Device-side errors of a run are reported by that run's next synchronising
 * call.  The lattice update is the row form (whole x rows
 * per wavefront) for runs with nx <= 256, else one node per thread, whatever
 * a run's IBM_OPT_LBM_VARIANT; the row form stores the first quarter of each
 * run's rows with cached writes and the rest non-temporally.  The stencil-box mode is the first run's
 * IBM_OPT_STENCIL_BOX if it was set, else 5 (box spreading, interpolation
 * from the node-velocity field) when the batch's membranes make at least 256
 * blocks of work, else 0. */
int ibm_batch_step(ibm_batch *b, int64_t n);

/* Tune the batch on its live runs by timing whole batched steps with HIP
 * events (each candidate: its graphs captured and replayed, then the better
 * of two timings over steps_per_trial steps, rounded up to a multiple of
 * 16): first the row-form lattice update's block shape (4, 2 or 1 wavefronts
 * of whole rows per block) and the fraction of each run's rows stored with
 * cached writes (1/4, 1/2 or none), then, for each delta width present, the
 * stencil-box mode of that width's runs (0, 1, 3 or 5, see
 * IBM_OPT_STENCIL_BOX), and last the persistent launch of
 * ibm_batch_set_persistent against the graphs of per-phase launches.  The
 * runs advance by all these steps (every candidate computes the same update,
 * to FP32 rounding).  chosen (nullable, 6 ints) receives the wavefronts per
 * block at index 0, the denominator of the cached fraction (0: none) at
 * index 1, the modes of delta widths 2, 3 and 4 at indices 2, 3 and 4 (-1 for
 * a width no run uses), and 1 at index 5 if the persistent launch was kept.
 * Waits. */
int ibm_batch_autotune(ibm_batch *b, int steps_per_trial, int *chosen);

/* on = 1: ibm_batch_step runs each step as one persistent launch (a
 * cooperative launch of as many blocks as the GPU holds at once, every phase
 * of every run in it, grid-wide barriers between spreading, the lattice
 * update, the velocity field and interpolation) instead of replaying graphs
 * of one launch per phase; used only when every run's rows fit the row form
 * (nx <= 256).  on = 0 (default): the per-phase launches.  Same results to
 * FP32 rounding. */
int ibm_batch_set_persistent(ibm_batch *b, int on);

/* ibm_profile_step for a batch: n steps of every run with plain launches and
 * HIP events between the batched kernels; ms_per_phase[IBM_N_PHASES] gets
 * the mean duration per step of each phase.  For measurement; waits. */
int ibm_batch_profile_step(ibm_batch *b, int64_t n, double *ms_per_phase);

/* ibm_profile_lattice_kernel for a batch: the mean execution time of the
 * batched collide-stream kernel over n steps of every run. */
int ibm_batch_profile_lattice_kernel(ibm_batch *b, int64_t n, double *ms);

/* Release the batch (not the runs or dev_mem); waits first. */
int ibm_batch_destroy(ibm_batch *b);

/* Thread-local description of the last error ("" if none). */
const char *ibm_last_error(void);

/* Icosahedron subdivided `level` times, nodes pushed radially onto the sphere
 * of radius r about (cx, cy, cz) (Sec. II.D, Fig. 3): nn = 10 * 4^level + 2
 * nodes, nf = 20 * 4^level faces, counter-clockwise seen from outside.
 * xyz host [nn][3], tri host [nf][3].  0 <= level <= 7. */
int ibm_icosphere_size(int level, int *nn, int *nf);
int ibm_icosphere(int level, double r, double cx, double cy, double cz,
                  double *xyz, int32_t *tri);

#ifdef __cplusplus
}
#endif

#endif /* IBM_LBM_H */
