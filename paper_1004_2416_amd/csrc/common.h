// Internal definitions shared by the kernels and the host runtime of the
// IB-LB-FEM library (arXiv:1004.2416).  Not part of the public ABI.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ibm {

constexpr int Q = 19;

// D3Q19 velocity set in the numbering of the paper's lattice sketch (Sec. II.A,
// Fig. 1): 1-6 along the axes, 7-18 along the face diagonals, 2k-1 and 2k
// opposite.  Indexed only with compile-time constants (fully unrolled loops).
__host__ __device__ constexpr int cx(int i) {
  constexpr int v[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, -1, 1, 1, -1, 0, 0, 0, 0};
  return v[i];
}
__host__ __device__ constexpr int cy(int i) {
  constexpr int v[Q] = {0, 0, 0, 1, -1, 0, 0, 0, 0, -1, 1, 0, 0, -1, 1, -1, 1, -1, 1};
  return v[i];
}
__host__ __device__ constexpr int cz(int i) {
  constexpr int v[Q] = {0, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1};
  return v[i];
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
// Lattice weights of D3Q19 (Qian et al., cited in Sec. II.A).
__host__ __device__ constexpr double wgt(int i) {
  return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// Force-density tiles of TILE_X x TILE_Y x TILE_Z lattice nodes.  Spreading
// stamps every tile it adds force to with the step number; the collide-stream
// kernel reads the force field only in tiles stamped with the current step
// and clears the other (previous step's) field where that one was stamped.
constexpr int TILE_X = 4, TILE_Y = 4, TILE_Z = 4;

// Device-side error flags (Ctrl::err bits).
constexpr int ERR_WALL = 1;      // a nonzero stencil weight beyond a wall
constexpr int ERR_FACE = 2;      // a face with non-positive deformed area
constexpr int ERR_NONFINITE = 4; // NaN/Inf in the observables
constexpr int ERR_SLAB = 8;      // a nonzero stencil weight outside [zlo, zhi)

struct alignas(256) Ctrl {
  int step;   // number of completed timesteps (incremented by the last kernel)
  int err;    // ERR_* bits, OR-ed by kernels, cleared by the host
  int zmin, zmax;  // lattice z and y extents of the membrane nodes (k_node_range)
  int ymin, ymax;
  int pad[58];
};

// Index of component c of node n in the force density fields L.g: the three
// components of a node are adjacent, so the spreading's atomic adds for a run
// of nodes along x cover one contiguous span (atomics cost per span they touch
// as well as per element), and the velocity pass finds a node's force in one
// cache line.
__host__ __device__ __forceinline__ long long gix(long long n, int c) { return 3 * n + c; }

// Everything the lattice kernels need, passed by value.
struct LatDev {
  int nx, ny, nz;
  int tnx, tny, tnz;      // tile grid
  long long S;            // stride between force-density components (elements)
  int gsh;                // log2 of the x rows per population group
  int nxs;                // population row stride: nx rounded up to a multiple of 4
  int tpr, rpw;           // row form: lanes per row (nxs / 4) and rows per
                          // wavefront (64 / tpr), or 0 where it does not apply
  int mass_fix;           // FP16 row form: the rest population takes back
                          // the mass the node's other values lose to
                          // rounding (fp16_mass_fix)
  int aa;                 // 1: the AA streaming pattern in buffer 0 (see
                          // collide_stream_rowseg_a); 0: two buffers
  int cached_rows;        // the row form writes the new populations of rows
                          // z ny + y below this with ordinary (cached) stores,
                          // the others with non-temporal ones
  void *f[2];             // population buffers (float or __half), see pidx
  float *g[2];            // force density of even and odd steps, [S][3]:
                          // the components of a node adjacent (gix)
  int *stamp[2];          // per-tile step stamps of the two fields
  int *nstamp;            // per node [S]: the last step whose stencils gave
                          // it a nonzero weight (the nodes interpolation reads)
  int zlo, zhi, ylo, yhi; // rows (z, y) stencils may reach: the whole lattice
                          // unless the update is split, see IBM_OPT_OVERLAP
  float4 *U;              // lattice velocity (ux, uy, uz, 0) at the nodes the
                          // step's stencils touch, for interpolation [S]
  Ctrl *ctrl;
  float inv_tau;          // 1 / tau
  float guo_pre;          // 1 - 1 / (2 tau)
  float uw;               // wall speed: top +uw, bottom -uw along x
  float h_scale[Q];       // FP16 storage: stored = (f_i - w_i) * h_scale[i]
  float h_inv[Q];         // 1 / h_scale[i], rounded to FP32
  long long pst[Q];       // i * pstride: offset of population i within a group
};

// A set of x rows (row = z ny + y) for the row-form lattice update: the run
// a0 .. a0 + n0 - 1, then n1 rows of the box z in [bz, ...), y in [by, by + wy)
// taken y fastest.
struct RowSet {
  int a0, n0, bz, by, wy, n1;
};
__device__ __forceinline__ int rowset_row(const RowSet &rs, const LatDev &L, int k) {
  if (k < rs.n0) return rs.a0 + k;
  k -= rs.n0;
  const int q = k / rs.wy;
  return (rs.bz + q) * L.ny + rs.by + (k - q * rs.wy);
}

// Membrane arrays (all capsules concatenated).
struct MemDev {
  int n_caps, nn, nf, m;
  float4 *x;        // node coordinates relative to the capsule origin [nn]
  float4 *u;        // node velocities of the last step [nn]
  float4 *F;        // nodal forces of the last step [nn]
  int *ext_id;      // caller's index of each (spatially sorted) node [nn]
  int *node_cap;    // capsule of each node [nn]
  int *csr_off;     // node -> incident (face, corner) list offsets [nn + 1]
  int *csr_ent;     // entries: face * 4 + corner [3 nf]
  int4 *tri;        // faces: global node ids a, b, c and capsule [nf]
  float4 *ref_p;    // inverse reference edge matrix (p, q, s) and area A0 [nf]
  float4 *ref_ghi;  // reference metric G0 = E0^T E0: (g11, g12, g22) high parts
  float4 *ref_glo;  // low parts (G0 - high), so hi + lo carries FP64 accuracy
  int4 *origin;     // integer frame origin of each capsule [n_caps]
  float4 *moduli;   // (k_s, k_alpha) per capsule [n_caps]
  int *cap_node_off;  // [n_caps + 1]
  int *cap_face_off;  // [n_caps + 1]
  double *obs;      // observables [n_caps][IBM_OBS_N]
  int cmode;        // batched runs: the coupling kernels' stencil-box mode
                    // (bits as IBM_OPT_STENCIL_BOX) chosen for this run
};

// Tangent-linear (forward sensitivity) state: the derivative of every
// evolving quantity along one parameter direction, advanced by the tangent
// kernels beside the timestep.
struct TanDev {
  float *df[2];   // tangent populations [19][S], same parity as the populations
  float *dg[2];   // tangent force density [3][S], same parity as the force field
  float4 *dx;     // tangent node positions [nn]
  float4 *du;     // tangent node velocities of the last step [nn]
  float4 *dF;     // tangent nodal forces of the last step [nn]
  float2 *dmod;   // (d k_s, d k_alpha) per capsule
  double *obs;    // [2][n_caps][16]: observables at x + h dx and at x - h dx
  float duw;      // d u_w (wall speed)
};

// Adjoint (reverse-mode) state of the timestep: the derivative of one scalar
// objective with respect to every quantity of the step being reversed.
struct AdjDev {
  float *lf[2];     // adjoints of the populations, same layout as the populations
  float *lU;        // adjoint of the lattice velocity at stencil nodes [3][S]
  float *lg;        // adjoint of the force density [3][S]
  float4 *lx;       // adjoint of the node positions [nn]
  float4 *lx_tmp;   // partial sums within one reverse step [nn]
  float4 *lF;       // adjoint of the nodal forces [nn]
  double2 *pk;      // per node: accumulated d/dk_s, d/dk_alpha of its capsule's moduli
  double *uw_col;   // per wall column (bottom, top) [2][ny][nx]: accumulated d/du_w
  int *stamp;       // per tile: the step whose stencils touched it (nonzero weight)
};

// Independent runs advanced together: every kernel of the step is launched once
// for all runs, each block working for one run.  Work items map a block to
// (run, block index within that run's own launch).
struct BatchDev {
  const LatDev *lat;       // [n_runs]
  const MemDev *mem;       // [n_runs]
  const int2 *lat_items;   // lattice update: 256 nodes per block, one per thread
  const int2 *node_items;  // spreading / interpolation: 256 / group_size lanes
  int n_lat_items, n_node_items;
  int wpb;                 // wavefronts per block of the row-form lattice update
  int any_field;           // some run interpolates from the node-velocity field
};

// Blocks of one run's batched lattice update (64 wpb threads each): the row
// form with wpb wavefronts of rpw whole rows each, else one node per thread.
__host__ __device__ inline long long batch_lat_blocks(const LatDev &L, int wpb) {
  const long long rows = (long long)L.ny * L.nz;
  if (L.tpr > 0) return ((rows + L.rpw - 1) / L.rpw + wpb - 1) / wpb;
  return ((long long)L.nx * rows + 64 * wpb - 1) / (64 * wpb);
}


// Lattice totals (ibm_lattice_totals): one FP64 partial sum (mass deviation,
// momentum) per TOTALS_NODES consecutive lattice nodes.
constexpr int TOTALS_NODES = 4096;

// ---- discrete delta functions, Sec. II.C Eqs. (2point), (3point), (4point) ----
// Evaluated for |r| inside the stencil; square-root arguments are clamped at 0
// so that rounding at the support edge cannot produce NaN.
template <int M>
__device__ __forceinline__ float phi(float r) {
  float a = fabsf(r);
  if constexpr (M == 2) {
    return fmaxf(1.0f - a, 0.0f);
  } else if constexpr (M == 3) {
    if (a <= 0.5f) return (1.0f + sqrtf(fmaxf(1.0f - 3.0f * a * a, 0.0f))) * (1.0f / 3.0f);
    if (a < 1.5f) return (5.0f - 3.0f * a - sqrtf(fmaxf(-2.0f + 6.0f * a - 3.0f * a * a, 0.0f))) * (1.0f / 6.0f);
    return 0.0f;
  } else {
    if (a <= 1.0f) return (3.0f - 2.0f * a + sqrtf(fmaxf(1.0f + 4.0f * a - 4.0f * a * a, 0.0f))) * 0.125f;
    if (a < 2.0f) return (5.0f - 2.0f * a - sqrtf(fmaxf(-7.0f + 12.0f * a - 4.0f * a * a, 0.0f))) * 0.125f;
    return 0.0f;
  }
}

// Derivatives d phi / dr of the three deltas (zero outside the support; the
// 2-point delta takes -sign(r), 0 at its kink r = 0).
template <int M>
__device__ __forceinline__ float dphi(float r) {
  const float a = fabsf(r);
  const float sg = r > 0.0f ? 1.0f : (r < 0.0f ? -1.0f : 0.0f);
  if constexpr (M == 2) {
    return a < 1.0f ? -sg : 0.0f;
  } else if constexpr (M == 3) {
    if (a <= 0.5f) return -r / sqrtf(fmaxf(1.0f - 3.0f * a * a, 1e-30f));
    if (a < 1.5f)
      return sg * (-0.5f - (1.0f - a) * 0.5f / sqrtf(fmaxf(-2.0f + 6.0f * a - 3.0f * a * a, 1e-30f)));
    return 0.0f;
  } else {
    if (a <= 1.0f)
      return sg * 0.25f * (-1.0f + (1.0f - 2.0f * a) / sqrtf(fmaxf(1.0f + 4.0f * a - 4.0f * a * a, 1e-30f)));
    if (a < 2.0f)
      return sg * 0.25f * (-1.0f - (3.0f - 2.0f * a) / sqrtf(fmaxf(-7.0f + 12.0f * a - 4.0f * a * a, 1e-30f)));
    return 0.0f;
  }
}

// First lattice coordinate of the M-point stencil around position p: the M
// integers within M/2 of p.
template <int M>
__device__ __forceinline__ int stencil_lo(float p) {
  if constexpr (M == 3) return (int)floorf(p + 0.5f) - 1;
  else if constexpr (M == 4) return (int)floorf(p) - 1;
  else return (int)floorf(p);
}

// Populations are stored interleaved by groups of G = 2^gsh x rows
// (row = z ny + y): [row / G][i][row % G][x], each x row padded to nxs (a
// multiple of 4) values.  Each population of a group is one contiguous run
// of G nxs values (G chosen so that G nxs >= 128 where possible), so an update
// reads and writes a few contiguous kilobytes per group instead of 19 arrays
// that are megabytes apart.  The padding (x >= nx) holds no lattice node.
// pidx(L, i, row, x) = prow(L, row) + i pstride(L) + x: a per-row offset and
// a stride between the populations of a group that is the same for all rows.
__host__ __device__ __forceinline__ long long prow(const LatDev &L, long long row) {
  const long long g = row >> L.gsh, r = row - (g << L.gsh);
  return (((g * Q) << L.gsh) + r) * (long long)L.nxs;
}
__host__ __device__ __forceinline__ long long pstride(const LatDev &L) {
  return (long long)L.nxs << L.gsh;
}
__host__ __device__ __forceinline__ long long pidx(const LatDev &L, int i, long long row, int x) {
  return prow(L, row) + i * pstride(L) + x;
}
// The same for a compile-time direction i: the offset of population i comes
// from the table (one 64-bit add per access instead of a multiply).
__host__ __device__ __forceinline__ long long pidx_c(const LatDev &L, int i, long long row, int x) {
  return prow(L, row) + L.pst[i] + x;
}

// Population storage geometry of an nx x ny x nz lattice: x rows padded to
// nxs, a multiple of 4 values (aligned 4-node vectors); 2^gsh rows per group,
// the smallest power of two (up to 8) whose group holds at least 128 values
// per population, so short rows still fill cache lines; the row form of the
// collide-stream kernel (tpr lanes per row, rpw rows per wavefront) where a
// padded row fits one wavefront and the padded row count times Q stays below
// 2^32 (its 32-bit group-row indices, see grow32), else tpr = rpw = 0.
struct PopGeometry {
  int nxs, gsh, tpr, rpw;
  long long pop_elems;  // elements of one population buffer
};
__host__ __device__ inline PopGeometry pop_geometry(int nx, int ny, int nz) {
  PopGeometry p{};
  p.nxs = (nx + 3) / 4 * 4;
  p.gsh = 0;
  while (p.gsh < 3 && ((long long)p.nxs << p.gsh) < 128) ++p.gsh;
  const long long g = 1LL << p.gsh;
  const long long rows = ((long long)ny * nz + g - 1) / g * g;
  p.pop_elems = (long long)Q * rows * p.nxs;
  p.tpr = (p.nxs / 4 <= 64 && rows * Q < (1LL << 32)) ? p.nxs / 4 : 0;
  p.rpw = p.tpr ? 64 / p.tpr : 0;
  return p;
}

__device__ __forceinline__ int wrap_mod(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

__device__ __forceinline__ int tile_of(const LatDev &L, int x, int y, int z) {
  return ((z / TILE_Z) * L.tny + (y / TILE_Y)) * L.tnx + (x / TILE_X);
}

// Lane-group size for the (membrane node, stencil node) mapping: the M^3
// stencil nodes of one membrane node occupy one power-of-two lane group.
template <int M>
__host__ __device__ constexpr int group_size() {
  return M == 2 ? 8 : (M == 3 ? 32 : 64);
}

}  // namespace ibm
