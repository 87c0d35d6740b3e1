// Membrane and coupling kernels: Skalak finite-element forces (Sec. II.B),
// force spreading and velocity interpolation with the discrete delta
// functions (Sec. II.C), Euler / Adams-Bashforth advection, FP64 reference
// geometry and shape observables (Sec. III).
//
// Node coordinates are FP32 relative to an integer origin per capsule, so a
// capsule of radius r keeps ~r * 2^-24 absolute resolution wherever it sits
// in the box.  Spreading and interpolation put the M^3 stencil nodes of one
// membrane node on one power-of-two lane group (8, 32 or 64 lanes).
#include <algorithm>

#include "common.h"
#include "launch.h"
#include "lbm_device.h"

#include <hip/hip_cooperative_groups.h>

namespace ibm {

// ---- finite-element forces ----------------------------------------------------

// Rounding error of s = a + b (Knuth's TwoSum); s must be fl(a + b).
__device__ __forceinline__ float two_sum_err(float a, float b, float s) {
#pragma clang fp contract(off)
  const float bb = s - a;
  return (a - (s - bb)) + (b - bb);
}

// Difference of two FP32 coordinates as an unevaluated sum hi + lo, exactly.
struct Edge {
  float hx, hy, hz, lx, ly, lz;
};

__device__ __forceinline__ Edge edge_exact(const float4 a, const float4 b) {
#pragma clang fp contract(off)
  Edge e;
  e.hx = b.x - a.x;
  e.hy = b.y - a.y;
  e.hz = b.z - a.z;
  e.lx = two_sum_err(b.x, -a.x, e.hx);
  e.ly = two_sum_err(b.y, -a.y, e.hy);
  e.lz = two_sum_err(b.z, -a.z, e.hz);
  return e;
}

// u.v - (hi0 + lo0) for exact edge vectors u, v, with the products and sums
// carried error-free (FMA product errors, TwoSum) and the first-order low
// parts added, so that the small metric change of a nearly undeformed face
// keeps FP32 relative accuracy instead of being lost to cancellation.
__device__ __forceinline__ float dot_minus_ref(const Edge &u, const Edge &v, float hi0,
                                               float lo0) {
#pragma clang fp contract(off)
  const float p0 = u.hx * v.hx, p1 = u.hy * v.hy, p2 = u.hz * v.hz;
  const float e0 = fmaf(u.hx, v.hx, -p0), e1 = fmaf(u.hy, v.hy, -p1), e2 = fmaf(u.hz, v.hz, -p2);
  const float s1 = p0 + p1;
  const float t1 = two_sum_err(p0, p1, s1);
  const float s2 = s1 + p2;
  const float t2 = two_sum_err(s1, p2, s2);
  const float cross = (u.hx * v.lx + u.hy * v.ly + u.hz * v.lz) +
                      (u.lx * v.hx + u.ly * v.hy + u.lz * v.hz);
  const float d = s2 - hi0;
  return d + (((((e0 + e1) + e2) + (t1 + t2)) + cross) - lo0);
}

// Gradient of the face energy A0 w_S (Sec. II.B, Eq. constitutivelaw) with
// respect to its corners a, b, c.  With current edges E = [b - a, c - a],
// the reference edge matrix P (E0 = B P in an orthonormal in-plane frame B),
// the deformation gradient F = E P^-1 and C = F^T F:
//   I1 = tr C - 2,  I2 = det C - 1,
//   dW/dE = 2 A0 E P^-1 [w1 1 + w2 adj C] P^-T,
//   w1 = dw/dI1 = (k_s/6)(I1 + 1),  w2 = dw/dI2 = (k_a I2 - k_s)/6.
// Everything is formed from C - 1 = P^-T (E^T E - E0^T E0) P^-1 so that no
// O(1) terms cancel: w1 1 + w2 adj C = (k_s I1 + k_a I2)/6 1 + w2 adj(C - 1).
struct FaceRef {
  float p, q, s, A0;       // P^-1 = [[p, q], [0, s]], reference area
  float g11, g12, g22;     // E0^T E0, high parts
  float l11, l12, l22;     // low parts
};

// Intermediate quantities of one face, shared by the gradient and its tangent.
struct FaceState {
  float e1x, e1y, e1z, e2x, e2y, e2z;  // current edges b - a, c - a
  float c11, c12, c22;                 // C - 1
  float I1, I2, kap;
  float T11, T12, T22;                 // P^-1 S P^-T
  float k2;                            // 2 A0
};

__device__ __forceinline__ FaceState skalak_state(const float4 a, const float4 b, const float4 c,
                                                  const FaceRef &R, float ks, float ka) {
  const Edge u = edge_exact(a, b), v = edge_exact(a, c);
  const float d11 = dot_minus_ref(u, u, R.g11, R.l11);
  const float d12 = dot_minus_ref(u, v, R.g12, R.l12);
  const float d22 = dot_minus_ref(v, v, R.g22, R.l22);
  FaceState F;
  F.e1x = u.hx;
  F.e1y = u.hy;
  F.e1z = u.hz;
  F.e2x = v.hx;
  F.e2y = v.hy;
  F.e2z = v.hz;
  const float p = R.p, q = R.q, s = R.s;
  F.c11 = p * p * d11;
  F.c12 = p * (q * d11 + s * d12);
  F.c22 = q * (q * d11 + s * d12) + s * (q * d12 + s * d22);
  F.I1 = F.c11 + F.c22;
  F.I2 = F.I1 + (F.c11 * F.c22 - F.c12 * F.c12);
  const float sig = (ks * F.I1 + ka * F.I2) * (1.0f / 6.0f);
  F.kap = (ka * F.I2 - ks) * (1.0f / 6.0f);
  const float S11 = sig + F.kap * F.c22, S22 = sig + F.kap * F.c11, S12 = -F.kap * F.c12;
  const float r1 = p * S11 + q * S12, r2 = p * S12 + q * S22;
  F.T11 = r1 * p + r2 * q;
  F.T12 = r2 * s;
  F.T22 = s * s * S22;
  F.k2 = 2.0f * R.A0;
  return F;
}

__device__ __forceinline__ void skalak_face_grad(const float4 a, const float4 b, const float4 c,
                                                 const FaceRef &R, float ks, float ka,
                                                 float3 &ga, float3 &gb, float3 &gc,
                                                 bool &degenerate) {
  const FaceState F = skalak_state(a, b, c, R, ks, ka);
  const float k2 = F.k2;
  gb = make_float3(k2 * (F.T11 * F.e1x + F.T12 * F.e2x), k2 * (F.T11 * F.e1y + F.T12 * F.e2y),
                   k2 * (F.T11 * F.e1z + F.T12 * F.e2z));
  gc = make_float3(k2 * (F.T12 * F.e1x + F.T22 * F.e2x), k2 * (F.T12 * F.e1y + F.T22 * F.e2y),
                   k2 * (F.T12 * F.e1z + F.T22 * F.e2z));
  ga = make_float3(-(gb.x + gc.x), -(gb.y + gc.y), -(gb.z + gc.z));
  degenerate = !(1.0f + F.I2 > 1e-6f);
}

// Forward derivative of the three corner gradients along corner displacements
// da, db, dc and modulus rates dks, dka: each quantity of skalak_state
// differentiated by the product rule (C - 1 is bilinear in the edges, the
// invariants are polynomials in C - 1, the stresses linear in the invariants).
__device__ __forceinline__ void skalak_face_grad_tangent(const float4 a, const float4 b,
                                                         const float4 c, const float4 da,
                                                         const float4 db, const float4 dc,
                                                         const FaceRef &R, float ks, float ka,
                                                         float dks, float dka, float3 &tga,
                                                         float3 &tgb, float3 &tgc) {
  const FaceState F = skalak_state(a, b, c, R, ks, ka);
  const float p = R.p, q = R.q, s = R.s;
  const float dux = db.x - da.x, duy = db.y - da.y, duz = db.z - da.z;
  const float dvx = dc.x - da.x, dvy = dc.y - da.y, dvz = dc.z - da.z;
  const float dd11 = 2.0f * (F.e1x * dux + F.e1y * duy + F.e1z * duz);
  const float dd12 = (dux * F.e2x + duy * F.e2y + duz * F.e2z) + (F.e1x * dvx + F.e1y * dvy + F.e1z * dvz);
  const float dd22 = 2.0f * (F.e2x * dvx + F.e2y * dvy + F.e2z * dvz);
  const float dc11 = p * p * dd11;
  const float dc12 = p * (q * dd11 + s * dd12);
  const float dc22 = q * (q * dd11 + s * dd12) + s * (q * dd12 + s * dd22);
  const float dI1 = dc11 + dc22;
  const float dI2 = dI1 + (dc11 * F.c22 + F.c11 * dc22 - 2.0f * F.c12 * dc12);
  const float dsig = (dks * F.I1 + ks * dI1 + dka * F.I2 + ka * dI2) * (1.0f / 6.0f);
  const float dkap = (dka * F.I2 + ka * dI2 - dks) * (1.0f / 6.0f);
  const float dS11 = dsig + dkap * F.c22 + F.kap * dc22;
  const float dS22 = dsig + dkap * F.c11 + F.kap * dc11;
  const float dS12 = -(dkap * F.c12 + F.kap * dc12);
  const float dr1 = p * dS11 + q * dS12, dr2 = p * dS12 + q * dS22;
  const float dT11 = dr1 * p + dr2 * q, dT12 = dr2 * s, dT22 = s * s * dS22;
  const float k2 = F.k2;
  tgb = make_float3(k2 * (dT11 * F.e1x + F.T11 * dux + dT12 * F.e2x + F.T12 * dvx),
                    k2 * (dT11 * F.e1y + F.T11 * duy + dT12 * F.e2y + F.T12 * dvy),
                    k2 * (dT11 * F.e1z + F.T11 * duz + dT12 * F.e2z + F.T12 * dvz));
  tgc = make_float3(k2 * (dT12 * F.e1x + F.T12 * dux + dT22 * F.e2x + F.T22 * dvx),
                    k2 * (dT12 * F.e1y + F.T12 * duy + dT22 * F.e2y + F.T22 * dvy),
                    k2 * (dT12 * F.e1z + F.T12 * duz + dT22 * F.e2z + F.T22 * dvz));
  tga = make_float3(-(tgb.x + tgc.x), -(tgb.y + tgc.y), -(tgb.z + tgc.z));
}

// Work items of the lane-group kernels are handed out so that each XCD (the
// hardware deals consecutive blocks to the 8 XCDs in turn) gets one contiguous
// range of the spatially sorted membrane nodes: neighbouring stencils then
// meet in the same L2.  Returns -1 for the padding blocks.
__device__ __forceinline__ int xcd_block(int nblocks_real) {
  const int per = (nblocks_real + 7) / 8;
  const int b = (int)blockIdx.x;
  const int logical = (b % 8) * per + b / 8;
  return logical < nblocks_real ? logical : -1;
}

static unsigned xcd_grid(long long blocks) { return (unsigned)(((blocks + 7) / 8) * 8); }

// Butterfly sum over a power-of-two lane group.
template <int GS>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
  for (int off = GS / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, GS);
  return v;
}

// Minimum and maximum over the 64 lanes of a wavefront (all active) with DPP
// lane moves: within quads, half rows, rows, then rows 1 and 3 take row 0's and
// row 2's last lane, and rows 2 and 3 lane 31; lane 63 ends with the result.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ int dpp_mov(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, ROWS, 0xf, false);
}
template <bool MAX>
__device__ __forceinline__ int wave_extreme(int v) {
  auto op = [](int a, int b) { return MAX ? max(a, b) : min(a, b); };
  v = op(v, dpp_mov<0xb1>(v));        // quad_perm [1,0,3,2]
  v = op(v, dpp_mov<0x4e>(v));        // quad_perm [2,3,0,1]
  v = op(v, dpp_mov<0x141>(v));       // row_half_mirror
  v = op(v, dpp_mov<0x140>(v));       // row_mirror
  v = op(v, dpp_mov<0x142, 0xa>(v));  // row_bcast:15
  v = op(v, dpp_mov<0x143, 0xc>(v));  // row_bcast:31
  return __builtin_amdgcn_readlane(v, 63);
}

// ---- spreading, Eq. (forcespreading) -------------------------------------------
// One lane group per membrane node: the group first forms the node's Skalak
// force from its incident faces (Sec. II.B), then each lane adds
// F_n delta(X - x_n) to one stencil node X of the force field of parity `par`
// (FP32 atomics; the field starts at zero, see the collide-stream kernel) and
// stamps X's tile with the step number.
// The block's M^3 contributions of 256 / GS membrane nodes are first summed
// in an LDS box spanning their stencils (when it has at most SPREAD_BOX
// lattice nodes; in fixed point, see SpreadLDS), then every touched box node
// is added to the global field once per component, consecutive threads on
// consecutive addresses.  Overlapping stencils of neighbouring nodes would
// otherwise send many atomics to the same addresses at once, which
// serialises them; spread over the box, the adds are distinct and coalesced.
// block_box: the bounding box of the block's nonzero-weight stencil nodes
// (unwrapped lattice coordinates): wave-level min / max with shuffles, then
// across the block's waves in LDS (the interpolation's box; spreading uses
// wave_box and block_box_slots below).  All threads of the block must call
// it.
struct Box {
  int x0, y0, z0, ex, ey, ez, V;
  bool fits;
  int amax;  // block_box_slots only
};

__device__ __forceinline__ Box block_box(int gx0, int gy0, int gz0, int gx1, int gy1, int gz1,
                                         bool has, int capacity, int *bb) {
  int v[6] = {has ? gx0 : 0x7fffffff, has ? gy0 : 0x7fffffff, has ? gz0 : 0x7fffffff,
              has ? gx1 : -0x7fffffff, has ? gy1 : -0x7fffffff, has ? gz1 : -0x7fffffff};
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      v[k] = min(v[k], __shfl_xor(v[k], off, 64));
      v[k + 3] = max(v[k + 3], __shfl_xor(v[k + 3], off, 64));
    }
  }
  if (threadIdx.x < 6) bb[threadIdx.x] = threadIdx.x < 3 ? 0x7fffffff : -0x7fffffff;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      atomicMin(&bb[k], v[k]);
      atomicMax(&bb[k + 3], v[k + 3]);
    }
  }
  __syncthreads();
  Box b;
  b.amax = 0;
  b.x0 = bb[0];
  b.y0 = bb[1];
  b.z0 = bb[2];
  b.ex = bb[3] - bb[0] + 1;
  b.ey = bb[4] - bb[1] + 1;
  b.ez = bb[5] - bb[2] + 1;
  b.fits = bb[0] <= bb[3] && (long long)b.ex * b.ey * b.ez <= capacity;
  b.V = b.fits ? b.ex * b.ey * b.ez : 0;
  return b;
}

// The same box, and the block's largest `amax` (bits of a non-negative float
// or NaN, which order as integers like the values, NaN above infinity),
// with one barrier.  wave_box: each wavefront reduces with DPP and writes its
// seven values to its own slots of `slots` ([4][8], at most four
// wavefronts).  block_box_slots, after a barrier: every thread combines the
// slots.  All threads of the block must call both.
__device__ __forceinline__ void wave_box(int gx0, int gy0, int gz0, int gx1, int gy1, int gz1,
                                         bool has, int amax, int *slots) {
  const int v0 = wave_extreme<false>(has ? gx0 : 0x7fffffff);
  const int v1 = wave_extreme<false>(has ? gy0 : 0x7fffffff);
  const int v2 = wave_extreme<false>(has ? gz0 : 0x7fffffff);
  const int v3 = wave_extreme<true>(has ? gx1 : -0x7fffffff);
  const int v4 = wave_extreme<true>(has ? gy1 : -0x7fffffff);
  const int v5 = wave_extreme<true>(has ? gz1 : -0x7fffffff);
  const int v6 = wave_extreme<true>(amax);
  if ((threadIdx.x & 63) == 0) {
    int *o = slots + 8 * (threadIdx.x >> 6);
    o[0] = v0;
    o[1] = v1;
    o[2] = v2;
    o[3] = v3;
    o[4] = v4;
    o[5] = v5;
    o[6] = v6;
  }
}

__device__ __forceinline__ Box block_box_slots(const int *slots, int capacity) {
  int e[7] = {slots[0], slots[1], slots[2], slots[3], slots[4], slots[5], slots[6]};
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
    const int *o = slots + 8 * w;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      e[k] = min(e[k], o[k]);
      e[k + 3] = max(e[k + 3], o[k + 3]);
    }
    e[6] = max(e[6], o[6]);
  }
  // the same in every lane: kept in scalar registers
#pragma unroll
  for (int k = 0; k < 7; ++k) e[k] = __builtin_amdgcn_readfirstlane(e[k]);
  Box b;
  b.amax = e[6];
  b.x0 = e[0];
  b.y0 = e[1];
  b.z0 = e[2];
  b.ex = e[3] - e[0] + 1;
  b.ey = e[4] - e[1] + 1;
  b.ez = e[5] - e[2] + 1;
  b.fits = e[0] <= e[3] && (long long)b.ex * b.ey * b.ez <= capacity;
  b.V = b.fits ? b.ex * b.ey * b.ez : 0;
  return b;
}

// Up to SPREAD_BOX lattice nodes per box; its tiles, counted in unwrapped
// coordinates, number at most (ceil(ex/4) + 1)(ceil(ey/4) + 1)(ceil(ez/4) + 1)
// <= 772 for ex ey ez <= 768.  The box sums are 64-bit fixed point (see
// spread_lanes): LDS float atomics measured slow here (a block's three adds
// per stencil node took as long as the rest of its LDS work together, plain
// or integer adds a small part of that), integer ones are fast, and the fixed
// point sum is exact whatever the order of the adds.  20.0 KB per block:
// eight blocks of 256 threads per compute unit.
constexpr int SPREAD_BOX = 768;
constexpr int SPREAD_BOX_TILES = 776;
struct SpreadLDS {
  unsigned long long box[3][SPREAD_BOX];  // two's complement fixed point
  unsigned char nflag[SPREAD_BOX];        // box nodes some stencil weights nonzero
  unsigned char tflag[SPREAD_BOX_TILES];
  int slots[4][8];                        // wave_box
};
static_assert(SPREAD_BOX % 4 == 0 && SPREAD_BOX_TILES % 4 == 0, "flags are cleared in words");
// Fixed point of the box sums: a block whose largest force component has
// magnitude below 2^e counts in units of 2^(e - SPREAD_FIX_BITS).  Every
// contribution w F (w <= 1) is then below 2^SPREAD_FIX_BITS units and the at
// most 512 of a block sum to below 2^61; each is represented to 2^-52 of the
// block's largest force, far below FP32's own rounding.
constexpr int SPREAD_FIX_BITS = 52;

// The capsule holding most of a block's nodes [first, first + count): a block
// that straddles the end of one capsule holds two compact patches far apart,
// so only the larger one goes through the block's LDS box (the other lanes
// work directly on the global fields).  Uniform across the block.
__device__ __forceinline__ int block_major_capsule(const MemDev &Mm, int first, int count) {
  if (first >= Mm.nn) return -1;
  const int last = min(first + count, Mm.nn) - 1;
  const int c0 = Mm.node_cap[first];
  const int end0 = Mm.cap_node_off[c0 + 1];
  if (end0 > last) return c0;
  return (end0 - first) >= (last + 1 - end0) ? c0 : Mm.node_cap[end0];
}

// Lanes per membrane node in spreading.  With HALF the wider deltas give each
// lane two stencil nodes (27 or 64 of them on 16 or 32 lanes), which halves
// the wavefronts of the launch and the idle lanes of the force evaluation; on
// large membranes that measured 3-6 % faster steps (128^3, the batched
// sweep), on a single 642-node capsule (300 wavefronts) 4 % slower.
template <int M, bool HALF>
__host__ __device__ constexpr int spread_group_size() {
  return M == 2 ? 8 : (HALF ? group_size<M>() / 2 : group_size<M>());
}
// BATCH: the batched kernels' lane groups (batch_group_size).
template <int M, bool HALF, bool BATCH>
__host__ __device__ constexpr int coupling_group_size() {
  return BATCH ? batch_group_size(M) : spread_group_size<M, HALF>();
}
// Interpolation from the node-velocity field gathers 16 bytes per stencil
// node: each lane takes two stencil nodes (4, 16 or 32 lanes per membrane
// node), which halves the wavefronts of that short, latency-bound launch.
template <int M>
__host__ __device__ constexpr int field_group_size() {
  return M == 2 ? 4 : group_size<M>() / 2;
}
// HALF where the full lane groups would make at least this many wavefronts
constexpr long long SPREAD_HALF_WAVES = 1024;

template <int M, bool BOX, bool HALF = true, bool BATCH = false>
__device__ __forceinline__ void spread_lanes(const LatDev &L, const MemDev &Mm, int par, int blk,
                                             SpreadLDS &sm) {
  constexpr int GS = coupling_group_size<M, HALF, BATCH>();
  constexpr int M3 = M * M * M;
  constexpr int PPL = (M3 + GS - 1) / GS;  // stencil nodes per lane
  const int lane = threadIdx.x & (GS - 1);
  const int node = (blk * (int)blockDim.x + (int)threadIdx.x) / GS;
  const bool live = node < Mm.nn;  // whole groups alike
  const int npb = (int)blockDim.x / GS;
  // The loads the stencil and the LDS box need do not depend on the force:
  // issued here, their dependent chains (node -> capsule -> origin, and the
  // block's major capsule) overlap the force's instead of following it.
  const int cap = live ? Mm.node_cap[node] : -1;
  const float4 p = live ? Mm.x[node] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  const int4 o = live ? Mm.origin[cap] : make_int4(0, 0, 0, 0);
  const int major = (BOX && Mm.n_caps > 1) ? block_major_capsule(Mm, blk * npb, npb) : cap;
  const int step = L.ctrl->step;
  if constexpr (BOX) {
    // the whole LDS box is cleared before its extent is known
    for (int c = threadIdx.x; c < 3 * SPREAD_BOX; c += blockDim.x) (&sm.box[0][0])[c] = 0ull;
    for (int c = threadIdx.x; c < SPREAD_BOX / 4; c += blockDim.x)
      reinterpret_cast<unsigned *>(sm.nflag)[c] = 0u;
    for (int c = threadIdx.x; c < SPREAD_BOX_TILES / 4; c += blockDim.x)
      reinterpret_cast<unsigned *>(sm.tflag)[c] = 0u;
  }
  // Eq. (forcefromenergy): F_n = -sum over the faces at n of d(A0 w_S)/dx_n,
  // one incident face per lane (each face is evaluated by each of its corners)
  float fx = 0.0f, fy = 0.0f, fz = 0.0f;
  if (live) {
    const int e0 = Mm.csr_off[node], e1 = Mm.csr_off[node + 1];
    for (int e = e0 + lane; e < e1; e += GS) {
      const int ent = Mm.csr_ent[e];
      const int j = ent >> 2, corner = ent & 3;
      const int4 tj = Mm.tri[j];
      const float4 rp = Mm.ref_p[j], gh = Mm.ref_ghi[j], gl = Mm.ref_glo[j];
      const float4 mod = Mm.moduli[tj.w];
      const FaceRef R{rp.x, rp.y, rp.z, rp.w, gh.x, gh.y, gh.z, gl.x, gl.y, gl.z};
      float3 ga, gb, gc;
      bool deg;
      skalak_face_grad(Mm.x[tj.x], Mm.x[tj.y], Mm.x[tj.z], R, mod.x, mod.y, ga, gb, gc, deg);
      if (deg) atomicOr(&L.ctrl->err, ERR_FACE);
      const float3 g = corner == 0 ? ga : (corner == 1 ? gb : gc);
      fx -= g.x;
      fy -= g.y;
      fz -= g.z;
    }
  }
  fx = group_sum<GS>(fx);
  fy = group_sum<GS>(fy);
  fz = group_sum<GS>(fz);
  if (live && lane == 0) Mm.F[node] = make_float4(fx, fy, fz, 0.0f);
  // the bits of the largest |component| (NaN stays NaN: compared as integers)
  const int fbits = max(max(__float_as_int(fabsf(fx)), __float_as_int(fabsf(fy))),
                        __float_as_int(fabsf(fz)));
  // this lane's stencil nodes lane, lane + GS, ..., in unwrapped lattice
  // coordinates
  int gx[PPL], gy[PPL], gz[PPL];
  float w[PPL];
#pragma unroll
  for (int q = 0; q < PPL; ++q) {
    gx[q] = gy[q] = gz[q] = 0;
    w[q] = 0.0f;
  }
  if (live) {
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      const int sidx = lane + q * GS;
      if (sidx >= M3) continue;
      const int lx = stencil_lo<M>(p.x) + sidx % M;
      const int ly = stencil_lo<M>(p.y) + (sidx / M) % M;
      const int lz = stencil_lo<M>(p.z) + sidx / (M * M);
      float wq = phi<M>((float)lx - p.x) * phi<M>((float)ly - p.y) * phi<M>((float)lz - p.z);
      gx[q] = o.x + lx;
      gy[q] = o.y + ly;
      gz[q] = o.z + lz;
      if (wq != 0.0f && (gz[q] < 0 || gz[q] >= L.nz)) {
        atomicOr(&L.ctrl->err, ERR_WALL);
        wq = 0.0f;
      }
      // a split lattice update assumes no force outside the rows zlo <= z < zhi,
      // ylo <= y < yhi (nothing to check where they are the whole lattice)
      if (wq != 0.0f && (L.zlo > 0 || L.zhi < L.nz || L.ylo > 0 || L.yhi < L.ny)) {
        const int Y = wrap_mod(gy[q], L.ny);
        if (gz[q] < L.zlo || gz[q] >= L.zhi || Y < L.ylo || Y >= L.yhi)
          atomicOr(&L.ctrl->err, ERR_SLAB);
      }
      w[q] = wq;
    }
  }
  float *g = L.g[par];
  if constexpr (!BOX) {
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      if (w[q] == 0.0f) continue;
      const int X = wrap_mod(gx[q], L.nx), Y = wrap_mod(gy[q], L.ny);
      const long long n = ((long long)gz[q] * L.ny + Y) * L.nx + X;
      unsafeAtomicAdd(g + gix(n, 0), w[q] * fx);
      unsafeAtomicAdd(g + gix(n, 1), w[q] * fy);
      unsafeAtomicAdd(g + gix(n, 2), w[q] * fz);
      L.stamp[par][tile_of(L, X, Y, gz[q])] = step;
      L.nstamp[n] = step;
    }
    return;
  }
  // the lane's own extent over its nonzero-weight stencil nodes, if its
  // capsule is the block's major one
  const bool inbox = Mm.n_caps == 1 || cap == major;
  bool has = false;
  int bx0 = 0, by0 = 0, bz0 = 0, bx1 = 0, by1 = 0, bz1 = 0;
#pragma unroll
  for (int q = 0; q < PPL; ++q) {
    if (w[q] == 0.0f || !inbox) continue;
    bx0 = has ? min(bx0, gx[q]) : gx[q];
    by0 = has ? min(by0, gy[q]) : gy[q];
    bz0 = has ? min(bz0, gz[q]) : gz[q];
    bx1 = has ? max(bx1, gx[q]) : gx[q];
    by1 = has ? max(by1, gy[q]) : gy[q];
    bz1 = has ? max(bz1, gz[q]) : gz[q];
    has = true;
  }
  wave_box(bx0, by0, bz0, bx1, by1, bz1, has, fbits, &sm.slots[0][0]);
  // one barrier orders the slots and the clearing of the box (at the start)
  // before their use
  __syncthreads();
  const Box b = block_box_slots(&sm.slots[0][0], SPREAD_BOX);
  // a block with a non-finite force goes through the per-lane path (which
  // carries it into the field as the FP32 atomics would)
  const bool fits = b.fits && b.amax <= 0x7f7fffff;
  const int x0 = b.x0, y0 = b.y0, z0 = b.z0, ex = b.ex, ey = b.ey;
  const int V = fits ? b.V : 0;
  int fe;
  (void)frexpf(__int_as_float(fits ? b.amax : 0), &fe);
  const double to_fix = ldexp(1.0, SPREAD_FIX_BITS - fe), from_fix = ldexp(1.0, fe - SPREAD_FIX_BITS);
  // the box's tiles in unwrapped coordinates (>> 2 floors negative ones too)
  const int tx0 = x0 >> 2, ty0 = y0 >> 2, tz0 = z0 >> 2;
  const int ntx = fits ? ((x0 + ex - 1) >> 2) - tx0 + 1 : 0;
  const int nty = fits ? ((y0 + ey - 1) >> 2) - ty0 + 1 : 0;
  const int NT = fits ? ntx * nty * (((z0 + b.ez - 1) >> 2) - tz0 + 1) : 0;
#pragma unroll
  for (int q = 0; q < PPL; ++q) {
    if (w[q] == 0.0f) continue;
    if (fits && inbox) {
      const int c = ((gz[q] - z0) * ey + (gy[q] - y0)) * ex + (gx[q] - x0);
      atomicAdd(&sm.box[0][c], (unsigned long long)__double2ll_rn((double)(w[q] * fx) * to_fix));
      atomicAdd(&sm.box[1][c], (unsigned long long)__double2ll_rn((double)(w[q] * fy) * to_fix));
      atomicAdd(&sm.box[2][c], (unsigned long long)__double2ll_rn((double)(w[q] * fz) * to_fix));
      sm.nflag[c] = 1;
      sm.tflag[(((gz[q] >> 2) - tz0) * nty + ((gy[q] >> 2) - ty0)) * ntx + ((gx[q] >> 2) - tx0)] = 1;
    } else {
      const int X = wrap_mod(gx[q], L.nx), Y = wrap_mod(gy[q], L.ny);
      const long long n = ((long long)gz[q] * L.ny + Y) * L.nx + X;
      unsafeAtomicAdd(g + gix(n, 0), w[q] * fx);
      unsafeAtomicAdd(g + gix(n, 1), w[q] * fy);
      unsafeAtomicAdd(g + gix(n, 2), w[q] * fz);
      L.stamp[par][tile_of(L, X, Y, gz[q])] = step;
      L.nstamp[n] = step;
    }
  }
  if (!fits) return;  // the whole block
  __syncthreads();
  // only in-range z received force (see above); every node a nonzero weight
  // touched is marked for interpolation, whatever its force.  One component
  // per thread, consecutive threads on consecutive addresses: the adds of a
  // run of box nodes along x fall into one contiguous span of the field.
  // where the box spans at most one period along x and y, its wrapped start
  // and one conditional subtraction give each node's wrapped position
  const bool one_period = ex <= L.nx && ey <= L.ny;
  const int wx0 = wrap_mod(x0, L.nx), wy0 = wrap_mod(y0, L.ny);
  for (int k = threadIdx.x; k < 3 * V; k += blockDim.x) {
    const int c = k / 3, comp = k - 3 * c;
    if (!sm.nflag[c]) continue;
    const float v = (float)((double)(long long)sm.box[comp][c] * from_fix);
    const int row = c / ex, cx = c - row * ex, plane = row / ey, cy = row - plane * ey;
    int X, Y;
    if (one_period) {
      X = wx0 + cx;
      X -= X >= L.nx ? L.nx : 0;
      Y = wy0 + cy;
      Y -= Y >= L.ny ? L.ny : 0;
    } else {
      X = wrap_mod(x0 + cx, L.nx);
      Y = wrap_mod(y0 + cy, L.ny);
    }
    const int Z = z0 + plane;
    const long long n = ((long long)Z * L.ny + Y) * L.nx + X;
    if (comp == 0) L.nstamp[n] = step;
    if (v != 0.0f) unsafeAtomicAdd(g + gix(n, comp), v);
  }
  // Every tile a nonzero weight touches, once per block.  Where nx or ny is
  // not a multiple of 4, the four wrapped positions of an unwrapped tile fall
  // into up to three tiles along that axis: stamp all of them.
  // an unwrapped tile is one tile of the lattice where nx and ny are
  // multiples of the tile size; its wrapped position follows from the box's
  // wrapped first tile where the box spans at most one period of tiles
  const bool whole_tiles = (L.nx % TILE_X) == 0 && (L.ny % TILE_Y) == 0;
  const bool one_tile_period = whole_tiles && ntx <= L.tnx && nty <= L.tny;
  const int wtx0 = wrap_mod(tx0, L.tnx), wty0 = wrap_mod(ty0, L.tny);
  for (int q = threadIdx.x; q < NT; q += blockDim.x) {
    if (!sm.tflag[q]) continue;
    const int row = q / ntx, qx = q - row * ntx, qz = row / nty, qy = row - qz * nty;
    const int ux = tx0 + qx, uy = ty0 + qy, uz = tz0 + qz;
    if (one_tile_period) {
      int tx = wtx0 + qx, ty = wty0 + qy;
      tx -= tx >= L.tnx ? L.tnx : 0;
      ty -= ty >= L.tny ? L.tny : 0;
      L.stamp[par][(uz * L.tny + ty) * L.tnx + tx] = step;
      continue;
    }
    if (whole_tiles) {
      L.stamp[par][(uz * L.tny + wrap_mod(uy, L.tny)) * L.tnx + wrap_mod(ux, L.tnx)] = step;
      continue;
    }
    int tx[3], ty[3], nxt = 0, nyt = 0;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int a = wrap_mod(4 * ux + d, L.nx) >> 2, c = wrap_mod(4 * uy + d, L.ny) >> 2;
      if (nxt == 0 || (tx[nxt - 1] != a && tx[0] != a)) tx[nxt < 3 ? nxt++ : 2] = a;
      if (nyt == 0 || (ty[nyt - 1] != c && ty[0] != c)) ty[nyt < 3 ? nyt++ : 2] = c;
    }
    for (int i = 0; i < nyt; ++i)
      for (int j = 0; j < nxt; ++j) L.stamp[par][(uz * L.tny + ty[i]) * L.tnx + tx[j]] = step;
  }
}

template <int M, bool BOX, bool HALF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_spread(LatDev L, MemDev Mm, int par, int nblocks) {
  __shared__ SpreadLDS sm;
  const int blk = xcd_block(nblocks);
  if (blk >= 0) spread_lanes<M, BOX, HALF>(L, Mm, par, blk, sm);
}

void launch_spread(const LatDev &L, const MemDev &M, int par, bool box, hipStream_t s) {
  if (M.nn <= 0) return;
  const int full = M.m == 2 ? group_size<2>() : (M.m == 3 ? group_size<3>() : group_size<4>());
  const bool half = (long long)M.nn * full / 64 >= SPREAD_HALF_WAVES;
  const int gs = M.m == 2 ? full : (half ? full / 2 : full);
  const long long lanes = (long long)M.nn * gs;
  const int nblocks = (int)((lanes + 255) / 256);
  const dim3 grid(xcd_grid(nblocks)), block(256);
#define IBM_LAUNCH_SPREAD(BX)                                                               \
  do {                                                                                      \
    if (M.m == 2) k_spread<2, BX, false><<<grid, block, 0, s>>>(L, M, par, nblocks);        \
    else if (M.m == 3 && half) k_spread<3, BX, true><<<grid, block, 0, s>>>(L, M, par, nblocks); \
    else if (M.m == 3) k_spread<3, BX, false><<<grid, block, 0, s>>>(L, M, par, nblocks);   \
    else if (half) k_spread<4, BX, true><<<grid, block, 0, s>>>(L, M, par, nblocks);        \
    else k_spread<4, BX, false><<<grid, block, 0, s>>>(L, M, par, nblocks);                 \
  } while (0)
  if (box) IBM_LAUNCH_SPREAD(true);
  else IBM_LAUNCH_SPREAD(false);
#undef IBM_LAUNCH_SPREAD
}

// ---- interpolation + advection, Eqs. (velocityinterpolation), (positionupdate)
// u(X, t+1) = (sum_i c_i f_i(X, t+1) + f(X, t)/2) / rho(X, t+1) at each stencil
// node, weighted and summed over the lane group; the group's first lane moves
// the node.  advect: 0 Euler; 1 Adams-Bashforth x += 3/2 u(t+1) - 1/2 u(t)
// with u(t) the stored velocity of the previous step.  One thread advances
// the device step counter, which no other thread of this kernel reads.
template <typename T>
__device__ __forceinline__ float ld_pop(const T *p, long long idx, float inv_scale);
template <>
__device__ __forceinline__ float ld_pop<float>(const float *p, long long idx, float) {
  return p[idx];
}
template <>
__device__ __forceinline__ float ld_pop<__half>(const __half *p, long long idx, float inv_scale) {
  return __half2float(p[idx]) * inv_scale;
}

// The post-stream population deviation f_i - w_i at node (X, Y, Z) in state
// 2, the AA pattern after an even step (f: buffer 0): the post-collision
// values sit in the opposite slots of the nodes they leave,
// f_i(X) = A[opp(i)][X - c_i], or A[i][X] less the wall term of opp(i) for a
// population coming back from a wall (collide_stream_rowseg_a).
template <typename T>
__device__ __forceinline__ float pop_swapped(const LatDev &L, const T *f, int i, int X, int Y, int Z) {
  const int zs = Z - cz(i);
  if (cz(i) != 0 && (zs < 0 || zs >= L.nz))
    return ld_pop<T>(f, pidx(L, i, (long long)Z * L.ny + Y, X), L.h_inv[i]) - wall_kick(opp(i), L.uw);
  const int xs = X - cx(i) < 0 ? L.nx - 1 : (X - cx(i) >= L.nx ? 0 : X - cx(i));
  const int ys = Y - cy(i) < 0 ? L.ny - 1 : (Y - cy(i) >= L.ny ? 0 : Y - cy(i));
  return ld_pop<T>(f, pidx(L, opp(i), (long long)zs * L.ny + ys, xs), L.h_inv[i]);
}

// Lattice velocity u(X, t+1) of Eq. (velocityinterpolation) from the
// post-stream populations at their own nodes of the buffer f (a state or a
// checkpoint of the adjoint).
template <typename T>
__device__ __forceinline__ float3 lattice_velocity_of(const LatDev &L, const T *f, const float *g,
                                                      int X, int Y, int Z) {
  const long long row = (long long)Z * L.ny + Y;
  const long long n = row * L.nx + X;
  float drho = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float d = ld_pop<T>(f, pidx(L, i, row, X), L.h_inv[i]);
    drho += d;
    if (cx(i)) jx += cx(i) * d;
    if (cy(i)) jy += cy(i) * d;
    if (cz(i)) jz += cz(i) * d;
  }
  const float inv_rho = 1.0f / (1.0f + drho);
  return make_float3((jx + 0.5f * g[gix(n, 0)]) * inv_rho, (jy + 0.5f * g[gix(n, 1)]) * inv_rho,
                     (jz + 0.5f * g[gix(n, 2)]) * inv_rho);
}

// Lattice velocity u(X, t+1) of Eq. (velocityinterpolation) at lattice node
// (X, Y, Z) in state 2 of the AA pattern (f: buffer 0, pop_swapped).
template <typename T>
__device__ __forceinline__ float3 lattice_velocity_swapped(const LatDev &L, const T *f,
                                                           const float *g, int X, int Y, int Z) {
  const long long n = ((long long)Z * L.ny + Y) * L.nx + X;
  float drho = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float d = pop_swapped<T>(L, f, i, X, Y, Z);
    drho += d;
    if (cx(i)) jx += cx(i) * d;
    if (cy(i)) jy += cy(i) * d;
    if (cz(i)) jz += cz(i) * d;
  }
  const float inv_rho = 1.0f / (1.0f + drho);
  return make_float3((jx + 0.5f * g[gix(n, 0)]) * inv_rho, (jy + 0.5f * g[gix(n, 1)]) * inv_rho,
                     (jz + 0.5f * g[gix(n, 2)]) * inv_rho);
}

// The lattice velocity u(X, t+1) of Eq. (velocityinterpolation) at every
// node that this step's stencils touch with a nonzero weight (node stamp =
// step), into L.U, from population buffer fsrc, or (SW) from state 2 of the
// AA pattern in buffer 0.  Each wavefront scans WN consecutive nodes (lattice
// order, x fastest) for marks and lists the marked ones in LDS in that order;
// the block's four lists, taken one after the other, are then evaluated by
// all 256 threads, so that neighbouring marked nodes share cache lines and
// the wavefronts share the work however the marks fall in the block's range
// (a block runs as few dependent rounds of loads as its count allows).  Each
// node is evaluated once, however many stencils overlap on it.  All 256
// threads of the block call it; the block covers nodes [n0, n1),
// n1 - n0 <= 4 WN.
// Single lattices: 256 nodes per block.  Many small blocks keep blocks in
// every phase (scan, gather) at once, so the memory system stays busy while
// others scan (measured on the dense suspension: 2048, 1024, 512 and 256 nodes
// per block, each faster than the one before).
constexpr int NODE_VELOCITY_WN = 64;
constexpr int NODE_VELOCITY_NODES = 4 * NODE_VELOCITY_WN;  // nodes per block
// Batched runs: a lattice-update work item covers at most 1024 nodes, so a
// run has at least N / 1024 items, and item k takes the run's nodes
// [1024 k, 1024 (k + 1)) in the velocity pass (the items past the run's
// last node return at once).  (Splitting an item over four blocks made the
// many idle blocks of the batch cost more than the smaller ranges gave.)
constexpr int BATCH_ITEM_NODES = 1024;
template <int WN>
struct VelocityLDS {
  int list[4 * WN];  // the wavefronts' lists, WN entries each
  int wcount[4];     // their lengths
};

template <typename T, bool SW, int WN>
__device__ __forceinline__ void node_velocity_range(const LatDev &L, int fsrc, int par,
                                                    long long n0, long long n1,
                                                    VelocityLDS<WN> &sm) {
  int *list = sm.list, *wcount = sm.wcount;
  const int step = L.ctrl->step;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int *wl = list + wave * WN;
  const long long w0 = n0 + (long long)wave * WN;
  int cnt = 0;
#pragma unroll
  for (int k = 0; k < WN / 64; ++k) {
    const long long n = w0 + k * 64 + lane;
    const bool marked = n < n1 && L.nstamp[n] == step;
    const unsigned long long mask = __ballot(marked);
    if (marked) wl[cnt + __popcll(mask & ((1ull << lane) - 1))] = k * 64 + lane;
    cnt += __popcll(mask);
  }
  if (lane == 0) wcount[wave] = cnt;
  __syncthreads();
  // position j of the block's list: entry j - c[w] of wavefront w's list,
  // where c[w] counts the entries of the wavefronts before w
  const int c1 = wcount[0], c2 = c1 + wcount[1], c3 = c2 + wcount[2], total = c3 + wcount[3];
  const float *g = L.g[par];
  const T *f = static_cast<const T *>(L.f[SW ? 0 : fsrc]);
  for (int j = (int)threadIdx.x; j < total; j += 256) {
    const int w = (j >= c1) + (j >= c2) + (j >= c3);
    const int before = w == 0 ? 0 : (w == 1 ? c1 : (w == 2 ? c2 : c3));
    const long long n = n0 + (long long)w * WN + list[w * WN + (j - before)];
    const long long row = n / L.nx;
    const int X = (int)(n - row * L.nx), Y = (int)(row % L.ny), Z = (int)(row / L.ny);
    const float3 u = SW ? lattice_velocity_swapped<T>(L, f, g, X, Y, Z)
                        : lattice_velocity_of<T>(L, f, g, X, Y, Z);
    L.U[n] = make_float4(u.x, u.y, u.z, 0.0f);
  }
}

// Single lattices.  FP32: each thread takes one node and evaluates it if it
// is marked (no lists: four wavefronts issuing their own gathers measured
// 0.9 % faster steps on the dense suspension than one wavefront issuing the
// block's compacted list); FP16 keeps the lists (1.4 % faster there).
template <typename T, bool SW>
__global__ __launch_bounds__(256) void k_node_velocity(LatDev L, int fsrc, int par) {
  const long long N = (long long)L.nx * L.ny * L.nz;
  const long long n0 = (long long)blockIdx.x * NODE_VELOCITY_NODES;
  if constexpr (sizeof(T) == 4) {
    static_assert(NODE_VELOCITY_NODES == 256, "one node per thread of a 256-thread block");
    const long long n = n0 + threadIdx.x;
    if (n >= N || L.nstamp[n] != L.ctrl->step) return;
    const long long row = n / L.nx;
    const int X = (int)(n - row * L.nx), Y = (int)(row % L.ny), Z = (int)(row / L.ny);
    const float *g = L.g[par];
    const T *f = static_cast<const T *>(L.f[SW ? 0 : fsrc]);
    const float3 u = SW ? lattice_velocity_swapped<T>(L, f, g, X, Y, Z) : lattice_velocity_of<T>(L, f, g, X, Y, Z);
    L.U[n] = make_float4(u.x, u.y, u.z, 0.0f);
  } else {
    __shared__ VelocityLDS<NODE_VELOCITY_WN> sm;
    node_velocity_range<T, SW, NODE_VELOCITY_WN>(L, fsrc, par, n0, min(N, n0 + NODE_VELOCITY_NODES), sm);
  }
}

// The lattice velocity is evaluated once per lattice node of the block's
// stencil box that a stencil touches with nonzero weight (consecutive threads
// on consecutive x: coalesced population reads; neighbouring nodes share most
// of their stencil nodes) and the lanes read it from LDS.  Blocks whose box
// has more than INTERP_BOX nodes read the populations per lane.
constexpr int INTERP_BOX = 1024;
struct InterpLDS {
  float box[3][INTERP_BOX];
  unsigned char mark[INTERP_BOX];
  int bb[6];
};

// UF: read the lattice velocity from L.U (filled by the node-velocity pass
// of this step) instead of evaluating it from the populations.
// HALF: two stencil nodes per lane for the wider deltas, as in spreading.
// BATCH: the batched kernels' lane groups (batch_group_size), as in spreading.
// FIELD: the lane groups of field_group_size (UF only).
template <typename T, int M, bool BOX, bool UF, bool HALF = false, bool BATCH = false,
          bool FIELD = false>
__device__ __forceinline__ void interp_lanes(const LatDev &L, const MemDev &Mm, int fsrc, int par,
                                             int advect, int blk, InterpLDS &sm) {
  static_assert(!FIELD || UF, "field lane groups read the velocity field");
  constexpr int GS = FIELD ? field_group_size<M>() : coupling_group_size<M, HALF, BATCH>();
  constexpr int M3 = M * M * M;
  constexpr int PPL = (M3 + GS - 1) / GS;  // stencil nodes per lane
  const int lane = threadIdx.x & (GS - 1);
  const int node = (blk * (int)blockDim.x + (int)threadIdx.x) / GS;
  const bool live = node < Mm.nn;  // whole groups alike
  float4 p = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  int gx[PPL], gy[PPL], gz[PPL];
  float w[PPL];
#pragma unroll
  for (int q = 0; q < PPL; ++q) {
    gx[q] = gy[q] = gz[q] = 0;
    w[q] = 0.0f;
  }
  const int cap = live ? Mm.node_cap[node] : -1;
  if (live) {
    p = Mm.x[node];
    const int4 o = Mm.origin[cap];
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      const int sidx = lane + q * GS;
      if (sidx >= M3) continue;
      const int lx = stencil_lo<M>(p.x) + sidx % M;
      const int ly = stencil_lo<M>(p.y) + (sidx / M) % M;
      const int lz = stencil_lo<M>(p.z) + sidx / (M * M);
      float wq = phi<M>((float)lx - p.x) * phi<M>((float)ly - p.y) * phi<M>((float)lz - p.z);
      gx[q] = o.x + lx;
      gy[q] = o.y + ly;
      gz[q] = o.z + lz;
      if (wq != 0.0f && (gz[q] < 0 || gz[q] >= L.nz)) {
        atomicOr(&L.ctrl->err, ERR_WALL);
        wq = 0.0f;
      }
      w[q] = wq;
    }
  }
  const T *f = static_cast<const T *>(L.f[fsrc]);
  const float *g = L.g[par];
  Box b{0, 0, 0, 1, 1, 1, 0, false};
  // the LDS box covers the stencils of the block's major capsule only (see
  // block_major_capsule); the other lanes read the populations themselves
  bool inbox = false;
  if constexpr (BOX && !UF) {
    const int npb = (int)blockDim.x / GS;
    inbox = Mm.n_caps == 1 || cap == block_major_capsule(Mm, blk * npb, npb);
    bool has = false;
    int bx0 = 0, by0 = 0, bz0 = 0, bx1 = 0, by1 = 0, bz1 = 0;
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      if (w[q] == 0.0f || !inbox) continue;
      bx0 = has ? min(bx0, gx[q]) : gx[q];
      by0 = has ? min(by0, gy[q]) : gy[q];
      bz0 = has ? min(bz0, gz[q]) : gz[q];
      bx1 = has ? max(bx1, gx[q]) : gx[q];
      by1 = has ? max(by1, gy[q]) : gy[q];
      bz1 = has ? max(bz1, gz[q]) : gz[q];
      has = true;
    }
    b = block_box(bx0, by0, bz0, bx1, by1, bz1, has, INTERP_BOX, sm.bb);
  }
  const bool fits = b.fits;
  const int x0 = b.x0, y0 = b.y0, z0 = b.z0, ex = b.ex, ey = b.ey;
  const int V = b.V;
  if constexpr (BOX && !UF) {
    for (int c = threadIdx.x; c < V; c += blockDim.x) sm.mark[c] = 0;
    __syncthreads();
    if (fits && inbox) {
#pragma unroll
      for (int q = 0; q < PPL; ++q)
        if (w[q] != 0.0f) sm.mark[((gz[q] - z0) * ey + (gy[q] - y0)) * ex + (gx[q] - x0)] = 1;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < V; c += blockDim.x) {
      if (!sm.mark[c]) continue;
      const float3 u = lattice_velocity_of<T>(L, f, g, wrap_mod(x0 + c % ex, L.nx),
                                              wrap_mod(y0 + (c / ex) % ey, L.ny), z0 + c / (ex * ey));
      sm.box[0][c] = u.x;
      sm.box[1][c] = u.y;
      sm.box[2][c] = u.z;
    }
    __syncthreads();
  }
  float ux = 0.0f, uy = 0.0f, uz = 0.0f;
#pragma unroll
  for (int q = 0; q < PPL; ++q) {
    if (w[q] == 0.0f) continue;
    float3 u;
    if constexpr (UF) {
      const float4 v =
          L.U[((long long)gz[q] * L.ny + wrap_mod(gy[q], L.ny)) * L.nx + wrap_mod(gx[q], L.nx)];
      u = make_float3(v.x, v.y, v.z);
    } else if (fits && inbox) {
      const int cell = ((gz[q] - z0) * ey + (gy[q] - y0)) * ex + (gx[q] - x0);
      u = make_float3(sm.box[0][cell], sm.box[1][cell], sm.box[2][cell]);
    } else {
      u = lattice_velocity_of<T>(L, f, g, wrap_mod(gx[q], L.nx), wrap_mod(gy[q], L.ny), gz[q]);
    }
    ux += w[q] * u.x;
    uy += w[q] * u.y;
    uz += w[q] * u.z;
  }
  ux = group_sum<GS>(ux);
  uy = group_sum<GS>(uy);
  uz = group_sum<GS>(uz);
  if (live && lane == 0) {
    if (advect == 1) {
      const float4 up = Mm.u[node];
      p.x += 1.5f * ux - 0.5f * up.x;
      p.y += 1.5f * uy - 0.5f * up.y;
      p.z += 1.5f * uz - 0.5f * up.z;
    } else {
      p.x += ux;
      p.y += uy;
      p.z += uz;
    }
    Mm.u[node] = make_float4(ux, uy, uz, 0.0f);
    Mm.x[node] = p;
  }
}

template <typename T, int M, bool BOX, bool HALF>
__global__ __launch_bounds__(256) void k_interp_advect(LatDev L, MemDev Mm, int fsrc, int par,
                                                       int advect, int nblocks) {
  __shared__ InterpLDS sm;
  if (blockIdx.x == 0 && threadIdx.x == 0) L.ctrl->step = L.ctrl->step + 1;
  const int blk = xcd_block(nblocks);
  if (blk >= 0) interp_lanes<T, M, BOX, false, HALF>(L, Mm, fsrc, par, advect, blk, sm);
}

// Interpolation from the node-velocity field.
template <typename T, int M>
__global__ __launch_bounds__(256) void k_interp_field(LatDev L, MemDev Mm, int fsrc, int par,
                                                      int advect, int nblocks) {
  __shared__ InterpLDS sm;
  if (blockIdx.x == 0 && threadIdx.x == 0) L.ctrl->step = L.ctrl->step + 1;
  const int blk = xcd_block(nblocks);
  if (blk >= 0) interp_lanes<T, M, false, true, false, false, true>(L, Mm, fsrc, par, advect, blk, sm);
}

void launch_interp_advect(const LatDev &L, const MemDev &M, int fp16, int fsrc, int par,
                          int advect, int mode, hipStream_t s) {
  if (M.nn <= 0) return;
  // state 2 of the AA pattern (after an even step) is read by the velocity
  // pass alone: the other forms would carry its gather in every kernel
  const bool swapped = fsrc == 2;
  if (swapped) mode = 2;
  const int gs = M.m == 2 ? group_size<2>() : (M.m == 3 ? group_size<3>() : group_size<4>());
  const long long lanes = (long long)M.nn * gs;
  const int nblocks = (int)((lanes + 255) / 256);
  const dim3 grid(xcd_grid(nblocks)), block(256);
  if (mode != 2) {
    // the lattice velocity from the populations, per stencil node or per block
    // in an LDS box; two stencil nodes per lane on large membranes, as in
    // spreading
    const bool half = M.m != 2 && lanes / 64 >= SPREAD_HALF_WAVES;
    const int nb = half ? (int)((lanes / 2 + 255) / 256) : nblocks;
    const dim3 gr(xcd_grid(nb));
#define IBM_LAUNCH_INTERP(T, BX)                                                                  \
  do {                                                                                            \
    if (M.m == 2) k_interp_advect<T, 2, BX, false><<<gr, block, 0, s>>>(L, M, fsrc, par, advect, nb); \
    else if (M.m == 3 && half)                                                                     \
      k_interp_advect<T, 3, BX, true><<<gr, block, 0, s>>>(L, M, fsrc, par, advect, nb);          \
    else if (M.m == 3) k_interp_advect<T, 3, BX, false><<<gr, block, 0, s>>>(L, M, fsrc, par, advect, nb); \
    else if (half) k_interp_advect<T, 4, BX, true><<<gr, block, 0, s>>>(L, M, fsrc, par, advect, nb); \
    else k_interp_advect<T, 4, BX, false><<<gr, block, 0, s>>>(L, M, fsrc, par, advect, nb);      \
  } while (0)
    if (fp16) {
      if (mode == 1) IBM_LAUNCH_INTERP(__half, true);
      else IBM_LAUNCH_INTERP(__half, false);
    } else {
      if (mode == 1) IBM_LAUNCH_INTERP(float, true);
      else IBM_LAUNCH_INTERP(float, false);
    }
#undef IBM_LAUNCH_INTERP
    return;
  }
  // the lattice velocity at the marked nodes, then the stencil sums from it
  const long long N = (long long)L.nx * L.ny * L.nz;
  const dim3 vgrid((unsigned)((N + NODE_VELOCITY_NODES - 1) / NODE_VELOCITY_NODES));
  const int fb = swapped ? 0 : fsrc;  // the stencil sums read the field only
  const int fgs = M.m == 2 ? field_group_size<2>() : (M.m == 3 ? field_group_size<3>() : field_group_size<4>());
  const int nbf = (int)(((long long)M.nn * fgs + 255) / 256);
  const dim3 fgrid(xcd_grid(nbf));
#define IBM_LAUNCH_INTERP_FIELD(T)                                                                  \
  do {                                                                                              \
    if (swapped) k_node_velocity<T, true><<<vgrid, block, 0, s>>>(L, 0, par);                       \
    else k_node_velocity<T, false><<<vgrid, block, 0, s>>>(L, fsrc, par);                           \
    if (M.m == 2) k_interp_field<T, 2><<<fgrid, block, 0, s>>>(L, M, fb, par, advect, nbf);         \
    else if (M.m == 3) k_interp_field<T, 3><<<fgrid, block, 0, s>>>(L, M, fb, par, advect, nbf);    \
    else k_interp_field<T, 4><<<fgrid, block, 0, s>>>(L, M, fb, par, advect, nbf);                \
  } while (0)
  if (fp16) IBM_LAUNCH_INTERP_FIELD(__half);
  else IBM_LAUNCH_INTERP_FIELD(float);
#undef IBM_LAUNCH_INTERP_FIELD
}

// ---- tangent (forward sensitivity) of spreading and interpolation ----------------
// With r = X - x_n and Phi(r) = phi(r_x) phi(r_y) phi(r_z), a node moving by dx
// changes its weight at X by -grad Phi(r) . dx, so
//   dg(X)  = sum_n [dF_n Phi(r) - F_n (grad Phi(r) . dx_n)]          (spreading)
//   du_n   = sum_X [du(X) Phi(r) - u(X) (grad Phi(r) . dx_n)]        (interpolation)
// with du(X) = (dj + dg/2 - u drho) / rho the derivative of the lattice velocity.
template <int M>
__device__ __forceinline__ void stencil_weight(const float4 p, const float4 dp, int lane, int &lx,
                                               int &ly, int &lz, float &w, float &dw) {
  lx = stencil_lo<M>(p.x) + lane % M;
  ly = stencil_lo<M>(p.y) + (lane / M) % M;
  lz = stencil_lo<M>(p.z) + lane / (M * M);
  const float rx = (float)lx - p.x, ry = (float)ly - p.y, rz = (float)lz - p.z;
  const float wx = phi<M>(rx), wy = phi<M>(ry), wz = phi<M>(rz);
  w = wx * wy * wz;
  dw = -(dphi<M>(rx) * wy * wz * dp.x + wx * dphi<M>(ry) * wz * dp.y + wx * wy * dphi<M>(rz) * dp.z);
}

template <int M>
__global__ __launch_bounds__(256) void k_tangent_spread(LatDev L, MemDev Mm, TanDev Tn, int par,
                                                        int nblocks) {
  constexpr int GS = group_size<M>();
  const int blk = xcd_block(nblocks);
  if (blk < 0) return;
  const int lane = threadIdx.x & (GS - 1);
  const int node = (blk * (int)blockDim.x + (int)threadIdx.x) / GS;
  if (node >= Mm.nn) return;  // whole groups leave together
  float fx = 0.0f, fy = 0.0f, fz = 0.0f;
  const int e0 = Mm.csr_off[node], e1 = Mm.csr_off[node + 1];
  for (int e = e0 + lane; e < e1; e += GS) {
    const int ent = Mm.csr_ent[e];
    const int j = ent >> 2, corner = ent & 3;
    const int4 tj = Mm.tri[j];
    const float4 rp = Mm.ref_p[j], gh = Mm.ref_ghi[j], gl = Mm.ref_glo[j];
    const float4 mod = Mm.moduli[tj.w];
    const float2 dmod = Tn.dmod[tj.w];
    const FaceRef R{rp.x, rp.y, rp.z, rp.w, gh.x, gh.y, gh.z, gl.x, gl.y, gl.z};
    float3 ta, tb, tc;
    skalak_face_grad_tangent(Mm.x[tj.x], Mm.x[tj.y], Mm.x[tj.z], Tn.dx[tj.x], Tn.dx[tj.y],
                             Tn.dx[tj.z], R, mod.x, mod.y, dmod.x, dmod.y, ta, tb, tc);
    const float3 t = corner == 0 ? ta : (corner == 1 ? tb : tc);
    fx -= t.x;
    fy -= t.y;
    fz -= t.z;
  }
  fx = group_sum<GS>(fx);
  fy = group_sum<GS>(fy);
  fz = group_sum<GS>(fz);
  if (lane == 0) Tn.dF[node] = make_float4(fx, fy, fz, 0.0f);
  if (lane >= M * M * M) return;
  int lx, ly, lz;
  float w, dw;
  stencil_weight<M>(Mm.x[node], Tn.dx[node], lane, lx, ly, lz, w, dw);
  if (w == 0.0f) return;
  const int4 o = Mm.origin[Mm.node_cap[node]];
  const int Z = o.z + lz;
  if (Z < 0 || Z >= L.nz) return;  // flagged by the spreading kernel
  const int X = wrap_mod(o.x + lx, L.nx), Y = wrap_mod(o.y + ly, L.ny);
  const long long n = ((long long)Z * L.ny + Y) * L.nx + X;
  const float4 F = Mm.F[node];
  float *dg = Tn.dg[par];
  unsafeAtomicAdd(dg + n, w * fx + dw * F.x);
  unsafeAtomicAdd(dg + L.S + n, w * fy + dw * F.y);
  unsafeAtomicAdd(dg + 2 * L.S + n, w * fz + dw * F.z);
}

template <int M>
__global__ __launch_bounds__(256) void k_tangent_interp(LatDev L, MemDev Mm, TanDev Tn, int fsrc,
                                                        int par, int nblocks) {
  constexpr int GS = group_size<M>();
  const int blk = xcd_block(nblocks);
  if (blk < 0) return;
  const int lane = threadIdx.x & (GS - 1);
  const int node = (blk * (int)blockDim.x + (int)threadIdx.x) / GS;
  if (node >= Mm.nn) return;  // whole groups leave together
  const float4 dp = Tn.dx[node];
  float ux = 0.0f, uy = 0.0f, uz = 0.0f;
  if (lane < M * M * M) {
    int lx, ly, lz;
    float w, dw;
    stencil_weight<M>(Mm.x[node], dp, lane, lx, ly, lz, w, dw);
    const int4 o = Mm.origin[Mm.node_cap[node]];
    const int Z = o.z + lz;
    if (w != 0.0f && Z >= 0 && Z < L.nz) {
      const int X = wrap_mod(o.x + lx, L.nx), Y = wrap_mod(o.y + ly, L.ny);
      const long long row = (long long)Z * L.ny + Y;
      const long long n = row * L.nx + X;
      const float *f = static_cast<const float *>(L.f[fsrc]);
      const float *df = Tn.df[fsrc];
      float drho = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
      float trho = 0.0f, tjx = 0.0f, tjy = 0.0f, tjz = 0.0f;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const float d = f[pidx(L, i, row, X)], t = df[i * L.S + n];
        drho += d;
        trho += t;
        if (cx(i)) {
          jx += cx(i) * d;
          tjx += cx(i) * t;
        }
        if (cy(i)) {
          jy += cy(i) * d;
          tjy += cy(i) * t;
        }
        if (cz(i)) {
          jz += cz(i) * d;
          tjz += cz(i) * t;
        }
      }
      const float *g = L.g[par], *dg = Tn.dg[par];
      const float inv_rho = 1.0f / (1.0f + drho);
      const float vx = (jx + 0.5f * g[gix(n, 0)]) * inv_rho;
      const float vy = (jy + 0.5f * g[gix(n, 1)]) * inv_rho;
      const float vz = (jz + 0.5f * g[gix(n, 2)]) * inv_rho;
      const float tvx = (tjx + 0.5f * dg[n] - vx * trho) * inv_rho;
      const float tvy = (tjy + 0.5f * dg[L.S + n] - vy * trho) * inv_rho;
      const float tvz = (tjz + 0.5f * dg[2 * L.S + n] - vz * trho) * inv_rho;
      ux = w * tvx + dw * vx;
      uy = w * tvy + dw * vy;
      uz = w * tvz + dw * vz;
    }
  }
  ux = group_sum<GS>(ux);
  uy = group_sum<GS>(uy);
  uz = group_sum<GS>(uz);
  if (lane == 0) {
    Tn.du[node] = make_float4(ux, uy, uz, 0.0f);
    Tn.dx[node] = make_float4(dp.x + ux, dp.y + uy, dp.z + uz, 0.0f);
  }
}

void launch_tangent_spread(const LatDev &L, const MemDev &M, const TanDev &T, int par,
                           hipStream_t s) {
  if (M.nn <= 0) return;
  const int gs = M.m == 2 ? group_size<2>() : (M.m == 3 ? group_size<3>() : group_size<4>());
  const int nblocks = (int)(((long long)M.nn * gs + 255) / 256);
  const dim3 grid(xcd_grid(nblocks)), block(256);
  if (M.m == 2) k_tangent_spread<2><<<grid, block, 0, s>>>(L, M, T, par, nblocks);
  else if (M.m == 3) k_tangent_spread<3><<<grid, block, 0, s>>>(L, M, T, par, nblocks);
  else k_tangent_spread<4><<<grid, block, 0, s>>>(L, M, T, par, nblocks);
}

void launch_tangent_interp(const LatDev &L, const MemDev &M, const TanDev &T, int fsrc, int par,
                           hipStream_t s) {
  if (M.nn <= 0) return;
  const int gs = M.m == 2 ? group_size<2>() : (M.m == 3 ? group_size<3>() : group_size<4>());
  const int nblocks = (int)(((long long)M.nn * gs + 255) / 256);
  const dim3 grid(xcd_grid(nblocks)), block(256);
  if (M.m == 2) k_tangent_interp<2><<<grid, block, 0, s>>>(L, M, T, fsrc, par, nblocks);
  else if (M.m == 3) k_tangent_interp<3><<<grid, block, 0, s>>>(L, M, T, fsrc, par, nblocks);
  else k_tangent_interp<4><<<grid, block, 0, s>>>(L, M, T, fsrc, par, nblocks);
}

// ---- adjoint (reverse mode) of the coupling and the membrane forces ---------------
// With r = X - x_n, Phi(r) = phi(r_x) phi(r_y) phi(r_z) and d Phi / d x_n =
// -grad Phi(r):
//   interpolation u_n = sum_X Phi U(X):   lU(X) += Phi lu_n,
//                                          lx_n  += -sum_X (U(X) . lu_n) grad Phi
//   spreading g(X) = sum_n Phi F_n:       lF_n   = sum_X Phi lg(X),
//                                          lx_n  += -sum_X (F_n . lg(X)) grad Phi
//   forces F = -grad W(x; k_s, k_alpha):   lx    += (dF/dx)^T lF = (dF/dx) lF
//                                          (the Hessian of W is symmetric, so the
//                                          tangent kernel's product serves),
//                                          d/dk_s += (dF/dk_s) . lF, likewise k_alpha.
// Advection x(t+1) = x(t) + u_n gives lu_n = lx(t+1) and lx(t) = lx(t+1) + ...
template <int M>
__global__ __launch_bounds__(256) void k_adj_interp(LatDev L, MemDev Mm, AdjDev A, const float *f1,
                                                    int par, int step, int nblocks) {
  constexpr int GS = group_size<M>();
  const int blk = xcd_block(nblocks);
  if (blk < 0) return;
  const int lane = threadIdx.x & (GS - 1);
  const int node = (blk * (int)blockDim.x + (int)threadIdx.x) / GS;
  if (node >= Mm.nn) return;  // whole groups leave together
  const float4 lu = A.lx[node];
  float gx = 0.0f, gy = 0.0f, gz = 0.0f;
  if (lane < M * M * M) {
    int lx, ly, lz;
    float w, dw;
    const float4 p = Mm.x[node];
    stencil_weight<M>(p, make_float4(0.0f, 0.0f, 0.0f, 0.0f), lane, lx, ly, lz, w, dw);
    const int4 o = Mm.origin[Mm.node_cap[node]];
    const int Z = o.z + lz;
    if (w != 0.0f && Z >= 0 && Z < L.nz) {
      const float rx = (float)lx - p.x, ry = (float)ly - p.y, rz = (float)lz - p.z;
      const float wx = phi<M>(rx), wy = phi<M>(ry), wz = phi<M>(rz);
      const float dx = dphi<M>(rx) * wy * wz, dy = wx * dphi<M>(ry) * wz, dz = wx * wy * dphi<M>(rz);
      const int X = wrap_mod(o.x + lx, L.nx), Y = wrap_mod(o.y + ly, L.ny);
      const float3 U = lattice_velocity_of<float>(L, f1, L.g[par], X, Y, Z);
      const float su = U.x * lu.x + U.y * lu.y + U.z * lu.z;
      gx = -su * dx;
      gy = -su * dy;
      gz = -su * dz;
      const long long n = ((long long)Z * L.ny + Y) * L.nx + X;
      A.stamp[tile_of(L, X, Y, Z)] = step;
      unsafeAtomicAdd(A.lU + n, w * lu.x);
      unsafeAtomicAdd(A.lU + L.S + n, w * lu.y);
      unsafeAtomicAdd(A.lU + 2 * L.S + n, w * lu.z);
    }
  }
  gx = group_sum<GS>(gx);
  gy = group_sum<GS>(gy);
  gz = group_sum<GS>(gz);
  if (lane == 0) A.lx_tmp[node] = make_float4(lu.x + gx, lu.y + gy, lu.z + gz, 0.0f);
}

template <int M>
__global__ __launch_bounds__(256) void k_adj_spread(LatDev L, MemDev Mm, AdjDev A, int nblocks) {
  constexpr int GS = group_size<M>();
  const int blk = xcd_block(nblocks);
  if (blk < 0) return;
  const int lane = threadIdx.x & (GS - 1);
  const int node = (blk * (int)blockDim.x + (int)threadIdx.x) / GS;
  if (node >= Mm.nn) return;  // whole groups leave together
  const float4 F = Mm.F[node];
  float fx = 0.0f, fy = 0.0f, fz = 0.0f, gx = 0.0f, gy = 0.0f, gz = 0.0f;
  if (lane < M * M * M) {
    int lx, ly, lz;
    float w, dw;
    const float4 p = Mm.x[node];
    stencil_weight<M>(p, make_float4(0.0f, 0.0f, 0.0f, 0.0f), lane, lx, ly, lz, w, dw);
    const int4 o = Mm.origin[Mm.node_cap[node]];
    const int Z = o.z + lz;
    if (w != 0.0f && Z >= 0 && Z < L.nz) {
      const float rx = (float)lx - p.x, ry = (float)ly - p.y, rz = (float)lz - p.z;
      const float wx = phi<M>(rx), wy = phi<M>(ry), wz = phi<M>(rz);
      const float dx = dphi<M>(rx) * wy * wz, dy = wx * dphi<M>(ry) * wz, dz = wx * wy * dphi<M>(rz);
      const int X = wrap_mod(o.x + lx, L.nx), Y = wrap_mod(o.y + ly, L.ny);
      const long long n = ((long long)Z * L.ny + Y) * L.nx + X;
      const float ax = A.lg[n], ay = A.lg[L.S + n], az = A.lg[2 * L.S + n];
      fx = w * ax;
      fy = w * ay;
      fz = w * az;
      const float sf = F.x * ax + F.y * ay + F.z * az;
      gx = -sf * dx;
      gy = -sf * dy;
      gz = -sf * dz;
    }
  }
  fx = group_sum<GS>(fx);
  fy = group_sum<GS>(fy);
  fz = group_sum<GS>(fz);
  gx = group_sum<GS>(gx);
  gy = group_sum<GS>(gy);
  gz = group_sum<GS>(gz);
  if (lane == 0) {
    A.lF[node] = make_float4(fx, fy, fz, 0.0f);
    const float4 t = A.lx_tmp[node];
    A.lx_tmp[node] = make_float4(t.x + gx, t.y + gy, t.z + gz, 0.0f);
  }
}

// Eight lanes per node, one incident face per lane.
__global__ __launch_bounds__(256) void k_adj_fem(LatDev L, MemDev Mm, AdjDev A, int nblocks) {
  constexpr int GS = 8;
  const int blk = xcd_block(nblocks);
  if (blk < 0) return;
  const int lane = threadIdx.x & (GS - 1);
  const int node = (blk * (int)blockDim.x + (int)threadIdx.x) / GS;
  if (node >= Mm.nn) return;  // whole groups leave together
  const float4 zero = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  float v[9] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  const int e1 = Mm.csr_off[node + 1];
  for (int e = Mm.csr_off[node] + lane; e < e1; e += GS) {
    const int ent = Mm.csr_ent[e];
    const int j = ent >> 2, corner = ent & 3;
    const int4 tj = Mm.tri[j];
    const float4 rp = Mm.ref_p[j], gh = Mm.ref_ghi[j], gl = Mm.ref_glo[j];
    const float4 mod = Mm.moduli[tj.w];
    const FaceRef R{rp.x, rp.y, rp.z, rp.w, gh.x, gh.y, gh.z, gl.x, gl.y, gl.z};
    const float4 a = Mm.x[tj.x], b = Mm.x[tj.y], c = Mm.x[tj.z];
    float3 t[3];
    // Hessian product with the force adjoints at the corners
    skalak_face_grad_tangent(a, b, c, A.lF[tj.x], A.lF[tj.y], A.lF[tj.z], R, mod.x, mod.y, 0.0f,
                             0.0f, t[0], t[1], t[2]);
    v[0] -= t[corner].x;
    v[1] -= t[corner].y;
    v[2] -= t[corner].z;
    // the face's corner force per unit k_s and per unit k_alpha
    skalak_face_grad_tangent(a, b, c, zero, zero, zero, R, mod.x, mod.y, 1.0f, 0.0f, t[0], t[1], t[2]);
    v[3] -= t[corner].x;
    v[4] -= t[corner].y;
    v[5] -= t[corner].z;
    skalak_face_grad_tangent(a, b, c, zero, zero, zero, R, mod.x, mod.y, 0.0f, 1.0f, t[0], t[1], t[2]);
    v[6] -= t[corner].x;
    v[7] -= t[corner].y;
    v[8] -= t[corner].z;
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) v[q] = group_sum<GS>(v[q]);
  if (lane == 0) {
    const float4 t = A.lx_tmp[node], lF = A.lF[node];
    A.lx[node] = make_float4(t.x + v[0], t.y + v[1], t.z + v[2], 0.0f);
    const double2 pk = A.pk[node];
    A.pk[node] = make_double2(pk.x + (double)(v[3] * lF.x + v[4] * lF.y + v[5] * lF.z),
                              pk.y + (double)(v[6] * lF.x + v[7] * lF.y + v[8] * lF.z));
  }
}

static int lanes_of(int m) {
  return m == 2 ? group_size<2>() : (m == 3 ? group_size<3>() : group_size<4>());
}

void launch_adj_interp(const LatDev &L, const MemDev &M, const AdjDev &A, const float *f1, int par,
                       int step, hipStream_t s) {
  if (M.nn <= 0) return;
  const int nblocks = (int)(((long long)M.nn * lanes_of(M.m) + 255) / 256);
  const dim3 grid(xcd_grid(nblocks)), block(256);
  if (M.m == 2) k_adj_interp<2><<<grid, block, 0, s>>>(L, M, A, f1, par, step, nblocks);
  else if (M.m == 3) k_adj_interp<3><<<grid, block, 0, s>>>(L, M, A, f1, par, step, nblocks);
  else k_adj_interp<4><<<grid, block, 0, s>>>(L, M, A, f1, par, step, nblocks);
}

void launch_adj_spread(const LatDev &L, const MemDev &M, const AdjDev &A, hipStream_t s) {
  if (M.nn <= 0) return;
  const int nblocks = (int)(((long long)M.nn * lanes_of(M.m) + 255) / 256);
  const dim3 grid(xcd_grid(nblocks)), block(256);
  if (M.m == 2) k_adj_spread<2><<<grid, block, 0, s>>>(L, M, A, nblocks);
  else if (M.m == 3) k_adj_spread<3><<<grid, block, 0, s>>>(L, M, A, nblocks);
  else k_adj_spread<4><<<grid, block, 0, s>>>(L, M, A, nblocks);
}

void launch_adj_fem(const LatDev &L, const MemDev &M, const AdjDev &A, hipStream_t s) {
  if (M.nn <= 0) return;
  const int nblocks = (int)(((long long)M.nn * 8 + 255) / 256);
  k_adj_fem<<<dim3(xcd_grid(nblocks)), dim3(256), 0, s>>>(L, M, A, nblocks);
}

// ---- batches of runs -------------------------------------------------------------
// Spreading (with the Skalak forces) and interpolation of many independent
// runs, one launch each; a block works for run items[b].x as block items[b].y of that
// run's own launch (so a block never mixes runs).  The delta width is chosen
// per block.
// Each run's spreading box (bit 0 of its cmode) is chosen per block.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_batch_spread(BatchDev B, int par) {
  __shared__ SpreadLDS sm;
  const int b = xcd_block(B.n_node_items);
  if (b < 0) return;
  const int2 it = B.node_items[b];
  const LatDev &L = B.lat[it.x];
  const MemDev &Mm = B.mem[it.x];
  const int m = Mm.m;
  if (Mm.cmode & 1) {
    if (m == 2) spread_lanes<2, true, true, true>(L, Mm, par, it.y, sm);
    else if (m == 3) spread_lanes<3, true, true, true>(L, Mm, par, it.y, sm);
    else spread_lanes<4, true, true, true>(L, Mm, par, it.y, sm);
  } else {
    if (m == 2) spread_lanes<2, false, true, true>(L, Mm, par, it.y, sm);
    else if (m == 3) spread_lanes<3, false, true, true>(L, Mm, par, it.y, sm);
    else spread_lanes<4, false, true, true>(L, Mm, par, it.y, sm);
  }
}

// The first block of each run advances that run's device step counter.  Each
// run's interpolation mode follows its cmode as for launch_interp_advect: per
// stencil node, per block in an LDS box (bit 1), or from the run's velocity
// field (bit 2; k_batch_node_velocity first).
template <typename T, int M>
__device__ __forceinline__ void batch_interp_m(const LatDev &L, const MemDev &Mm, int fsrc, int par,
                                               int advect, int blk, InterpLDS &sm) {
  if (Mm.cmode & 4) interp_lanes<T, M, false, true, true, true>(L, Mm, fsrc, par, advect, blk, sm);
  else if (Mm.cmode & 2) interp_lanes<T, M, true, false, true, true>(L, Mm, fsrc, par, advect, blk, sm);
  else interp_lanes<T, M, false, false, true, true>(L, Mm, fsrc, par, advect, blk, sm);
}

template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_batch_interp(BatchDev B, int fsrc, int par, int advect) {
  __shared__ InterpLDS sm;
  const int b = xcd_block(B.n_node_items);
  if (b < 0) return;
  const int2 it = B.node_items[b];
  const LatDev &L = B.lat[it.x];
  const MemDev &Mm = B.mem[it.x];
  if (it.y == 0 && threadIdx.x == 0) L.ctrl->step = L.ctrl->step + 1;
  const int m = Mm.m;
  if (m == 2) batch_interp_m<T, 2>(L, Mm, fsrc, par, advect, it.y, sm);
  else if (m == 3) batch_interp_m<T, 3>(L, Mm, fsrc, par, advect, it.y, sm);
  else batch_interp_m<T, 4>(L, Mm, fsrc, par, advect, it.y, sm);
}

// The velocity pass of every run, on the lattice work items: item k of a
// run takes its nodes [k, k + 1) * BATCH_ITEM_NODES.
template <typename T>
__global__ __launch_bounds__(256) void k_batch_node_velocity(BatchDev B, int fsrc, int par) {
  __shared__ VelocityLDS<BATCH_ITEM_NODES / 4> sm;
  if ((int)blockIdx.x >= B.n_lat_items) return;
  const int2 it = B.lat_items[blockIdx.x];
  const LatDev &L = B.lat[it.x];
  // no capsule (nothing is marked), or a run interpolating otherwise
  if (!B.mem[it.x].nn || !(B.mem[it.x].cmode & 4)) return;
  const long long N = (long long)L.nx * L.ny * L.nz;
  const long long n0 = (long long)it.y * BATCH_ITEM_NODES;
  if (n0 >= N) return;  // uniform across the block
  node_velocity_range<T, false, BATCH_ITEM_NODES / 4>(L, fsrc, par, n0, min(N, n0 + BATCH_ITEM_NODES), sm);
}

void launch_batch_spread(const BatchDev &B, int par, hipStream_t s) {
  if (B.n_node_items <= 0) return;
  const dim3 grid(xcd_grid(B.n_node_items)), block(256);
  k_batch_spread<<<grid, block, 0, s>>>(B, par);
}

void launch_batch_interp(const BatchDev &B, int fp16, int fsrc, int par, int advect, hipStream_t s) {
  if (B.n_node_items <= 0) return;
  const dim3 grid(xcd_grid(B.n_node_items)), block(256);
  if (fp16) {
    if (B.any_field) k_batch_node_velocity<__half><<<dim3(B.n_lat_items), block, 0, s>>>(B, fsrc, par);
    k_batch_interp<__half><<<grid, block, 0, s>>>(B, fsrc, par, advect);
  } else {
    if (B.any_field) k_batch_node_velocity<float><<<dim3(B.n_lat_items), block, 0, s>>>(B, fsrc, par);
    k_batch_interp<float><<<grid, block, 0, s>>>(B, fsrc, par, advect);
  }
}

// ---- the batched step as one persistent launch ------------------------------------
// One launch of co-resident blocks per step of every run (cooperative launch):
// the four phases (spreading, lattice update, velocity field, interpolation)
// each take all runs' work items, strided over the blocks, and grid-wide
// barriers separate them.  Only batches whose runs all use the row form.
// A grid barrier makes every block's writes visible across the XCDs' L2
// caches (an agent-scope release and acquire per block), the price of this
// form against separate launches.
template <typename T, bool LINEAR>
__device__ __forceinline__ void batch_cs_item(const BatchDev &B, int2 it, int src, int par) {
  LatDev L = B.lat[it.x];
  if (src) {
    void *t = L.f[0];
    L.f[0] = L.f[1];
    L.f[1] = t;
  }
  if (par) {
    float *tg = L.g[0];
    L.g[0] = L.g[1];
    L.g[1] = tg;
    int *ts = L.stamp[0];
    L.stamp[0] = L.stamp[1];
    L.stamp[1] = ts;
  }
  const int lane = threadIdx.x & 63;
  const int wave = it.y * B.wpb + (int)(threadIdx.x >> 6);
  if (wave * L.rpw >= L.ny * L.nz) return;  // the whole wavefront is past the last row
  const int r = lane / L.tpr;
  const int t = lane - r * L.tpr;
  const int row = wave * L.rpw + r;
  collide_stream_rowseg<T, LINEAR, true, true>(L, 0, 0, row, t, lane, r < L.rpw && row < L.ny * L.nz,
                                               __builtin_amdgcn_readfirstlane(row) < L.cached_rows);
}

template <typename T, bool LINEAR>
__global__ __launch_bounds__(256) void k_batch_persistent(BatchDev B, int src, int par, int advect) {
  // the phases, separated by grid barriers, share one LDS allocation
  __shared__ union {
    SpreadLDS s;
    InterpLDS i;
    VelocityLDS<BATCH_ITEM_NODES / 4> v;
  } sm;
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  for (int b = blockIdx.x; b < B.n_node_items; b += gridDim.x) {
    const int2 it = B.node_items[b];
    const LatDev &L = B.lat[it.x];
    const MemDev &Mm = B.mem[it.x];
    const int m = Mm.m;
    if (Mm.cmode & 1) {
      if (m == 2) spread_lanes<2, true, true, true>(L, Mm, par, it.y, sm.s);
      else if (m == 3) spread_lanes<3, true, true, true>(L, Mm, par, it.y, sm.s);
      else spread_lanes<4, true, true, true>(L, Mm, par, it.y, sm.s);
    } else {
      if (m == 2) spread_lanes<2, false, true, true>(L, Mm, par, it.y, sm.s);
      else if (m == 3) spread_lanes<3, false, true, true>(L, Mm, par, it.y, sm.s);
      else spread_lanes<4, false, true, true>(L, Mm, par, it.y, sm.s);
    }
    __syncthreads();  // the LDS box is reused by the next item
  }
  grid.sync();
  for (int b = blockIdx.x; b < B.n_lat_items; b += gridDim.x)
    batch_cs_item<T, LINEAR>(B, B.lat_items[b], src, par);
  grid.sync();
  if (B.any_field) {
    for (int b = blockIdx.x; b < B.n_lat_items; b += gridDim.x) {
      const int2 it = B.lat_items[b];
      const LatDev &L = B.lat[it.x];
      if (!B.mem[it.x].nn || !(B.mem[it.x].cmode & 4)) continue;  // uniform across the block
      const long long N = (long long)L.nx * L.ny * L.nz;
      const long long n0 = (long long)it.y * BATCH_ITEM_NODES;  // the item's whole range
      if (n0 >= N) continue;
      node_velocity_range<T, false, BATCH_ITEM_NODES / 4>(L, src ^ 1, par, n0,
                                                          min(N, n0 + BATCH_ITEM_NODES), sm.v);
      __syncthreads();  // the node lists are reused by the next item
    }
    grid.sync();
  }
  for (int b = blockIdx.x; b < B.n_node_items; b += gridDim.x) {
    const int2 it = B.node_items[b];
    const LatDev &L = B.lat[it.x];
    const MemDev &Mm = B.mem[it.x];
    if (it.y == 0 && threadIdx.x == 0) L.ctrl->step = L.ctrl->step + 1;
    const int m = Mm.m;
    if (m == 2) batch_interp_m<T, 2>(L, Mm, src ^ 1, par, advect, it.y, sm.i);
    else if (m == 3) batch_interp_m<T, 3>(L, Mm, src ^ 1, par, advect, it.y, sm.i);
    else batch_interp_m<T, 4>(L, Mm, src ^ 1, par, advect, it.y, sm.i);
    __syncthreads();
  }
}

template <typename T, bool LINEAR>
static int launch_batch_persistent_t(const BatchDev &B, int src, int par, int advect, hipStream_t s) {
  static int blocks = 0;  // co-resident blocks of this instantiation (per process)
  if (!blocks) {
    int per_cu = 0, cus = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_persistent<T, LINEAR>, 256, 0) !=
            hipSuccess || per_cu < 1)
      return -1;
    blocks = per_cu * cus;
  }
  BatchDev b = B;
  void *args[] = {&b, &src, &par, &advect};
  return hipLaunchCooperativeKernel(reinterpret_cast<void *>(k_batch_persistent<T, LINEAR>),
                                    dim3(blocks), dim3(256), args, 0, s) == hipSuccess ? 0 : -1;
}

int launch_batch_persistent(const BatchDev &B, int fp16, int src, int par, int advect, bool linear,
                            hipStream_t s) {
  if (fp16) {
    if (linear) return launch_batch_persistent_t<__half, true>(B, src, par, advect, s);
    return launch_batch_persistent_t<__half, false>(B, src, par, advect, s);
  }
  if (linear) return launch_batch_persistent_t<float, true>(B, src, par, advect, s);
  return launch_batch_persistent_t<float, false>(B, src, par, advect, s);
}

// ---- coupling kernels carrying part of a split lattice update -------------------
// IBM_OPT_OVERLAP: the lattice update of the x rows outside the force slab
// needs no force density, so it rides along with a coupling kernel.  Blocks
// [0, xcd_grid(nblocks)) of the launch do the coupling kernel's work; the
// blocks after them update the rows of rs in buffer fsrc into fsrc ^ 1 (row
// form, four wavefronts of whole rows per block).  The latency-bound coupling
// blocks and the bandwidth-bound lattice blocks then share the chip within
// one launch.
__device__ __forceinline__ int coupling_blocks(int nblocks) { return (nblocks + 7) / 8 * 8; }

template <typename T, bool LINEAR>
__device__ __forceinline__ void far_rows_block(const LatDev &L, int fsrc, int kb, const RowSet &rs) {
  const int lane = threadIdx.x & 63;
  const int wave = kb * 4 + (int)(threadIdx.x >> 6);
  const int n = rs.n0 + rs.n1;
  if (wave * L.rpw >= n) return;  // the whole wavefront is past the set
  const int r = lane / L.tpr;
  const int t = lane - r * L.tpr;
  const int k = wave * L.rpw + r;
  const bool live = r < L.rpw && k < n;
  collide_stream_rowseg<T, LINEAR, false, true>(L, fsrc, 0, live ? rowset_row(rs, L, k) : 0, t, lane,
                                                live, L.cached_rows != 0);
}

template <int M, bool BOX, typename T, bool LINEAR>
__global__ __launch_bounds__(256) void k_spread_far(LatDev L, MemDev Mm, int par, int nblocks,
                                                    int fsrc, RowSet rs) {
  __shared__ SpreadLDS sm;
  const int cb = coupling_blocks(nblocks);
  if ((int)blockIdx.x < cb) {
    const int blk = xcd_block(nblocks);
    if (blk >= 0) spread_lanes<M, BOX>(L, Mm, par, blk, sm);
    return;
  }
  far_rows_block<T, LINEAR>(L, fsrc, (int)blockIdx.x - cb, rs);
}

template <typename T, int M, int MODE, bool LINEAR>
__global__ __launch_bounds__(256) void k_interp_far(LatDev L, MemDev Mm, int fsrc, int par,
                                                    int advect, int nblocks, RowSet rs) {
  __shared__ InterpLDS sm;
  const int cb = coupling_blocks(nblocks);
  if ((int)blockIdx.x < cb) {
    if (blockIdx.x == 0 && threadIdx.x == 0) L.ctrl->step = L.ctrl->step + 1;
    const int blk = xcd_block(nblocks);
    if (blk >= 0) interp_lanes<T, M, MODE == 1, MODE == 2, true>(L, Mm, fsrc, par, advect, blk, sm);
    return;
  }
  far_rows_block<T, LINEAR>(L, fsrc, (int)blockIdx.x - cb, rs);
}

static unsigned far_blocks(const LatDev &L, const RowSet &rs) {
  const long long rows = (long long)rs.n0 + rs.n1;
  if (rows <= 0 || L.tpr <= 0) return 0;
  return (unsigned)(((rows + L.rpw - 1) / L.rpw + 3) / 4);
}

template <typename T, bool LINEAR>
static void launch_spread_far_t(const LatDev &L, const MemDev &M, int par, bool box, int fsrc,
                                const RowSet &rs, hipStream_t s) {
  const int gs = M.m == 2 ? spread_group_size<2, true>()
                          : (M.m == 3 ? spread_group_size<3, true>() : spread_group_size<4, true>());
  const int nblocks = (int)(((long long)M.nn * gs + 255) / 256);
  const dim3 grid(xcd_grid(nblocks) + far_blocks(L, rs)), block(256);
#define IBM_LAUNCH_SPREAD_FAR(BX)                                                                        \
  do {                                                                                                   \
    if (M.m == 2) k_spread_far<2, BX, T, LINEAR><<<grid, block, 0, s>>>(L, M, par, nblocks, fsrc, rs);      \
    else if (M.m == 3) k_spread_far<3, BX, T, LINEAR><<<grid, block, 0, s>>>(L, M, par, nblocks, fsrc, rs); \
    else k_spread_far<4, BX, T, LINEAR><<<grid, block, 0, s>>>(L, M, par, nblocks, fsrc, rs);          \
  } while (0)
  if (box) IBM_LAUNCH_SPREAD_FAR(true);
  else IBM_LAUNCH_SPREAD_FAR(false);
#undef IBM_LAUNCH_SPREAD_FAR
}

void launch_spread_far(const LatDev &L, const MemDev &M, int par, bool box, int fp16, bool linear,
                       int fsrc, const RowSet &rs, hipStream_t s) {
  if (M.nn <= 0) return;
  if (fp16) {
    if (linear) launch_spread_far_t<__half, true>(L, M, par, box, fsrc, rs, s);
    else launch_spread_far_t<__half, false>(L, M, par, box, fsrc, rs, s);
  } else {
    if (linear) launch_spread_far_t<float, true>(L, M, par, box, fsrc, rs, s);
    else launch_spread_far_t<float, false>(L, M, par, box, fsrc, rs, s);
  }
}

template <typename T, bool LINEAR>
static void launch_interp_far_t(const LatDev &L, const MemDev &M, int fsrc, int par, int advect,
                                int mode, const RowSet &rs, hipStream_t s) {
  const int gs = M.m == 2 ? spread_group_size<2, true>()
                          : (M.m == 3 ? spread_group_size<3, true>() : spread_group_size<4, true>());
  const int nblocks = (int)(((long long)M.nn * gs + 255) / 256);
  const dim3 grid(xcd_grid(nblocks) + far_blocks(L, rs)), block(256);
  if (mode == 2) {
    const long long N = (long long)L.nx * L.ny * L.nz;
    k_node_velocity<T, false><<<dim3((unsigned)((N + NODE_VELOCITY_NODES - 1) / NODE_VELOCITY_NODES)),
                                block, 0, s>>>(L, fsrc, par);
  }
#define IBM_LAUNCH_INTERP_FAR(MD)                                                                                \
  do {                                                                                                           \
    if (M.m == 2) k_interp_far<T, 2, MD, LINEAR><<<grid, block, 0, s>>>(L, M, fsrc, par, advect, nblocks, rs);      \
    else if (M.m == 3) k_interp_far<T, 3, MD, LINEAR><<<grid, block, 0, s>>>(L, M, fsrc, par, advect, nblocks, rs); \
    else k_interp_far<T, 4, MD, LINEAR><<<grid, block, 0, s>>>(L, M, fsrc, par, advect, nblocks, rs);          \
  } while (0)
  if (mode == 2) IBM_LAUNCH_INTERP_FAR(2);
  else if (mode == 1) IBM_LAUNCH_INTERP_FAR(1);
  else IBM_LAUNCH_INTERP_FAR(0);
#undef IBM_LAUNCH_INTERP_FAR
}

void launch_interp_far(const LatDev &L, const MemDev &M, int fp16, int fsrc, int par, int advect,
                       int mode, bool linear, const RowSet &rs, hipStream_t s) {
  if (M.nn <= 0) return;
  if (fp16) {
    if (linear) launch_interp_far_t<__half, true>(L, M, fsrc, par, advect, mode, rs, s);
    else launch_interp_far_t<__half, false>(L, M, fsrc, par, advect, mode, rs, s);
  } else {
    if (linear) launch_interp_far_t<float, true>(L, M, fsrc, par, advect, mode, rs, s);
    else launch_interp_far_t<float, false>(L, M, fsrc, par, advect, mode, rs, s);
  }
}

// ---- lattice extent of the membrane -------------------------------------------
__global__ __launch_bounds__(256) void k_node_range(MemDev M, Ctrl *ctrl) {
  int zlo = 0x7fffffff, zhi = -0x7fffffff, ylo = 0x7fffffff, yhi = -0x7fffffff;
  for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < M.nn; n += gridDim.x * blockDim.x) {
    const int4 o = M.origin[M.node_cap[n]];
    const float4 p = M.x[n];
    const int z = o.z + (int)floorf(p.z), y = o.y + (int)floorf(p.y);
    zlo = min(zlo, z);
    zhi = max(zhi, z);
    ylo = min(ylo, y);
    yhi = max(yhi, y);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    zlo = min(zlo, __shfl_xor(zlo, off, 64));
    zhi = max(zhi, __shfl_xor(zhi, off, 64));
    ylo = min(ylo, __shfl_xor(ylo, off, 64));
    yhi = max(yhi, __shfl_xor(yhi, off, 64));
  }
  // across the block's wavefronts, then four atomics per block (few blocks:
  // thousands of atomics on the same four words serialise)
  __shared__ int red[4][4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = zlo;
    red[1][w] = zhi;
    red[2][w] = ylo;
    red[3][w] = yhi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (int)(blockDim.x >> 6);
    for (int k = 1; k < nw; ++k) {
      zlo = min(zlo, red[0][k]);
      zhi = max(zhi, red[1][k]);
      ylo = min(ylo, red[2][k]);
      yhi = max(yhi, red[3][k]);
    }
    atomicMin(&ctrl->zmin, zlo);
    atomicMax(&ctrl->zmax, zhi);
    atomicMin(&ctrl->ymin, ylo);
    atomicMax(&ctrl->ymax, yhi);
  }
}

void launch_node_range(const MemDev &M, Ctrl *ctrl, hipStream_t s) {
  launch_fill_u32(&ctrl->zmin, 1, 0x7fffffffu, s);
  launch_fill_u32(&ctrl->zmax, 1, 0x80000001u, s);  // -0x7fffffff
  launch_fill_u32(&ctrl->ymin, 1, 0x7fffffffu, s);
  launch_fill_u32(&ctrl->ymax, 1, 0x80000001u, s);
  if (M.nn <= 0) return;
  const int blocks = (int)std::min<long long>(64, ((long long)M.nn + 255) / 256);
  k_node_range<<<dim3(blocks), dim3(256), 0, s>>>(M, ctrl);
}

// ---- capsule frame re-centring -------------------------------------------------
// Shift each capsule's integer origin towards its node centroid (and the FP32
// coordinates by the opposite integer) once the centroid has drifted by more
// than 1.5 lattice spacings; positions are unchanged up to FP32 rounding.
__global__ __launch_bounds__(256) void k_recenter(MemDev M) {
  __shared__ float red[3][256];
  __shared__ int shift[3];
  const int c = blockIdx.x;
  const int n0 = M.cap_node_off[c], n1 = M.cap_node_off[c + 1];
  float sx = 0.0f, sy = 0.0f, sz = 0.0f;
  for (int n = n0 + threadIdx.x; n < n1; n += blockDim.x) {
    const float4 p = M.x[n];
    sx += p.x;
    sy += p.y;
    sz += p.z;
  }
  red[0][threadIdx.x] = sx;
  red[1][threadIdx.x] = sy;
  red[2][threadIdx.x] = sz;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k)
      for (int d = 0; d < 3; ++d) red[d][threadIdx.x] += red[d][threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float inv = 1.0f / (float)(n1 - n0 > 0 ? n1 - n0 : 1);
    for (int d = 0; d < 3; ++d) {
      const float mean = red[d][0] * inv;
      shift[d] = fabsf(mean) > 1.5f ? (int)rintf(mean) : 0;
    }
  }
  __syncthreads();
  const int s0 = shift[0], s1 = shift[1], s2 = shift[2];
  if ((s0 | s1 | s2) == 0) return;
  for (int n = n0 + threadIdx.x; n < n1; n += blockDim.x) {
    float4 p = M.x[n];
    p.x -= (float)s0;
    p.y -= (float)s1;
    p.z -= (float)s2;
    M.x[n] = p;
  }
  if (threadIdx.x == 0) {
    int4 o = M.origin[c];
    o.x += s0;
    o.y += s1;
    o.z += s2;
    M.origin[c] = o;
  }
}

void launch_recenter(const MemDev &M, hipStream_t s) {
  if (M.n_caps <= 0) return;
  k_recenter<<<dim3(M.n_caps), dim3(256), 0, s>>>(M);
}

// ---- reference geometry (FP64) --------------------------------------------------
// Per face from the stored (exactly representable) initial coordinates: the
// in-plane reference edge matrix P = [[|e1|, e1.e2/|e1|], [0, |e1 x e2|/|e1|]],
// its inverse, the area A0 = |e1 x e2| / 2 and the metric E0^T E0 split into
// FP32 high and low parts.
__global__ __launch_bounds__(256) void k_reference_geometry(MemDev M, Ctrl *ctrl) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M.nf) return;
  const int4 t = M.tri[j];
  const float4 a = M.x[t.x], b = M.x[t.y], c = M.x[t.z];
  const double e1x = (double)b.x - a.x, e1y = (double)b.y - a.y, e1z = (double)b.z - a.z;
  const double e2x = (double)c.x - a.x, e2y = (double)c.y - a.y, e2z = (double)c.z - a.z;
  const double g11 = e1x * e1x + e1y * e1y + e1z * e1z;
  const double g12 = e1x * e2x + e1y * e2y + e1z * e2z;
  const double g22 = e2x * e2x + e2y * e2y + e2z * e2z;
  const double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
  const double area2 = sqrt(nx * nx + ny * ny + nz * nz);
  const double l1 = sqrt(g11);
  if (!(area2 > 1e-12 * g11) || !(l1 > 0.0)) {
    atomicOr(&ctrl->err, ERR_FACE);
    M.ref_p[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    return;
  }
  const double P11 = l1, P12 = g12 / l1, P22 = area2 / l1;
  M.ref_p[j] = make_float4((float)(1.0 / P11), (float)(-P12 / (P11 * P22)), (float)(1.0 / P22),
                           (float)(0.5 * area2));
  const float h11 = (float)g11, h12 = (float)g12, h22 = (float)g22;
  M.ref_ghi[j] = make_float4(h11, h12, h22, 0.0f);
  M.ref_glo[j] = make_float4((float)(g11 - h11), (float)(g12 - h12), (float)(g22 - h22), 0.0f);
}

void launch_reference_geometry(const MemDev &M, Ctrl *ctrl, hipStream_t s) {
  if (M.nf <= 0) return;
  k_reference_geometry<<<dim3((M.nf + 255) / 256), dim3(256), 0, s>>>(M, ctrl);
}

// ---- observables (FP64), Sec. III -------------------------------------------------

// Symmetric 3x3 eigen-decomposition by Jacobi rotations on the largest
// off-diagonal element.  a is overwritten; eigenvectors in the columns of v.
__device__ void sym3_eigen(double a[3][3], double v[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) v[i][j] = (i == j) ? 1.0 : 0.0;
  for (int it = 0; it < 60; ++it) {
    int p = 0, q = 1;
    double big = fabs(a[0][1]);
    if (fabs(a[0][2]) > big) { p = 0; q = 2; big = fabs(a[0][2]); }
    if (fabs(a[1][2]) > big) { p = 1; q = 2; big = fabs(a[1][2]); }
    const double diag = fabs(a[0][0]) + fabs(a[1][1]) + fabs(a[2][2]);
    if (big <= 1e-18 * diag || big == 0.0) break;
    const double th = 0.5 * atan2(2.0 * a[p][q], a[q][q] - a[p][p]);
    const double c = cos(th), s = sin(th);
    for (int k = 0; k < 3; ++k) {  // columns p, q of a
      const double akp = a[k][p], akq = a[k][q];
      a[k][p] = c * akp - s * akq;
      a[k][q] = s * akp + c * akq;
    }
    for (int k = 0; k < 3; ++k) {  // rows p, q
      const double apk = a[p][k], aqk = a[q][k];
      a[p][k] = c * apk - s * aqk;
      a[q][k] = s * apk + c * aqk;
    }
    for (int k = 0; k < 3; ++k) {
      const double vkp = v[k][p], vkq = v[k][q];
      v[k][p] = c * vkp - s * vkq;
      v[k][q] = s * vkp + c * vkq;
    }
  }
}

template <int K>
__device__ void block_sum(double (*red)[256], double *vals) {
  for (int k = 0; k < K; ++k) red[k][threadIdx.x] = vals[k];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < K; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  for (int k = 0; k < K; ++k) vals[k] = red[k][0];
  __syncthreads();
}

// One block per capsule.  Volume V = sum (a . (b x c))/6 and the volume
// centroid from signed tetrahedra; I = (1/5) sum_faces A (r^2 1 - r r)(r . n)
// with r the face centroid relative to the volume centroid, per unit mass
// (divided by V); the ellipsoid with that tensor has
// r_a^2 = 5/2 (E2 + E3 - E1), r_b^2 = 5/2 (E1 + E3 - E2),
// r_c^2 = 5/2 (E1 + E2 - E3) for eigenvalues E1 <= E2 <= E3.
// Node positions of the observables: stored coordinates, or x + h dx along a
// tangent, or one node moved by h along one axis.
struct PosShift {
  const MemDev *M;
  const float4 *dx;
  double h;
  __device__ __forceinline__ double3 operator()(int n) const {
    const float4 p = M->x[n];
    if (!dx) return make_double3(p.x, p.y, p.z);
    const float4 d = dx[n];
    return make_double3((double)p.x + h * d.x, (double)p.y + h * d.y, (double)p.z + h * d.z);
  }
};

struct PosPoke {
  const MemDev *M;
  int node, axis;
  double h;
  __device__ __forceinline__ double3 operator()(int n) const {
    const float4 p = M->x[n];
    double3 r = make_double3(p.x, p.y, p.z);
    if (n == node) {
      if (axis == 0) r.x += h;
      else if (axis == 1) r.y += h;
      else r.z += h;
    }
    return r;
  }
};

// Observables of capsule c (layout of ibm_observables, capsule-local
// centroid); all threads of the block call it, thread 0 gets out[] and the
// return value (all observables finite).
// aux (nullable, thread 0): the intermediates the derivative of D needs:
// [0] V, [1..6] the face sums S of I = S / (5 V) (xx, yy, zz, xy, xz, yz),
// [7..9] the eigenvalues E1 <= E2 <= E3, [10..18] their unit eigenvectors
// (v_k at 10 + 3k).
template <class Pos>
__device__ bool capsule_obs(const MemDev &M, int c, const Pos &pos, double (*red)[256], double *cen,
                            double *out, double *aux = nullptr) {
  const int f0 = M.cap_face_off[c], f1 = M.cap_face_off[c + 1];
  double v1[4] = {0.0, 0.0, 0.0, 0.0};
  for (int j = f0 + threadIdx.x; j < f1; j += blockDim.x) {
    const int4 t = M.tri[j];
    const double3 A = pos(t.x), B = pos(t.y), C = pos(t.z);
    const double ax = A.x, ay = A.y, az = A.z, bx = B.x, by = B.y, bz = B.z;
    const double cx_ = C.x, cy_ = C.y, cz_ = C.z;
    const double vt =
        (ax * (by * cz_ - bz * cy_) + ay * (bz * cx_ - bx * cz_) + az * (bx * cy_ - by * cx_)) / 6.0;
    v1[0] += vt;
    v1[1] += vt * (ax + bx + cx_) * 0.25;
    v1[2] += vt * (ay + by + cy_) * 0.25;
    v1[3] += vt * (az + bz + cz_) * 0.25;
  }
  block_sum<4>(red, v1);
  const double V = v1[0];
  if (threadIdx.x == 0) {
    cen[0] = v1[1] / V;
    cen[1] = v1[2] / V;
    cen[2] = v1[3] / V;
  }
  __syncthreads();
  double s7[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int j = f0 + threadIdx.x; j < f1; j += blockDim.x) {
    const int4 t = M.tri[j];
    const double3 A = pos(t.x), B = pos(t.y), C = pos(t.z);
    const double e1x = B.x - A.x, e1y = B.y - A.y, e1z = B.z - A.z;
    const double e2x = C.x - A.x, e2y = C.y - A.y, e2z = C.z - A.z;
    const double anx = 0.5 * (e1y * e2z - e1z * e2y);
    const double any = 0.5 * (e1z * e2x - e1x * e2z);
    const double anz = 0.5 * (e1x * e2y - e1y * e2x);
    const double rx = (A.x + B.x + C.x) / 3.0 - cen[0];
    const double ry = (A.y + B.y + C.y) / 3.0 - cen[1];
    const double rz = (A.z + B.z + C.z) / 3.0 - cen[2];
    const double rn = rx * anx + ry * any + rz * anz;
    const double r2 = rx * rx + ry * ry + rz * rz;
    s7[0] += (r2 - rx * rx) * rn;
    s7[1] += (r2 - ry * ry) * rn;
    s7[2] += (r2 - rz * rz) * rn;
    s7[3] += -rx * ry * rn;
    s7[4] += -rx * rz * rn;
    s7[5] += -ry * rz * rn;
    s7[6] += sqrt(anx * anx + any * any + anz * anz);
  }
  block_sum<7>(red, s7);
  bool finite = true;
  if (threadIdx.x == 0) {
    const double k = 1.0 / (5.0 * V);
    double I[6];
    for (int q = 0; q < 6; ++q) I[q] = s7[q] * k;
    double a[3][3] = {{I[0], I[3], I[4]}, {I[3], I[1], I[5]}, {I[4], I[5], I[2]}};
    double vec[3][3];
    sym3_eigen(a, vec);
    double e[3] = {a[0][0], a[1][1], a[2][2]};
    int id[3] = {0, 1, 2};
    for (int i = 0; i < 3; ++i)
      for (int j = i + 1; j < 3; ++j)
        if (e[id[j]] < e[id[i]]) {
          const int tmp = id[i];
          id[i] = id[j];
          id[j] = tmp;
        }
    const double E1 = e[id[0]], E2 = e[id[1]], E3 = e[id[2]];
    const double ra = sqrt(fmax(2.5 * (E2 + E3 - E1), 0.0));
    const double rb = sqrt(fmax(2.5 * (E1 + E3 - E2), 0.0));
    const double rc = sqrt(fmax(2.5 * (E1 + E2 - E3), 0.0));
    double th = atan2(vec[2][id[0]], vec[0][id[0]]);
    if (th <= -M_PI / 2) th += M_PI;
    if (th > M_PI / 2) th -= M_PI;
    if (!((E2 - E1) > 1e-12 * fabs(E3))) th = __longlong_as_double(0x7ff8000000000000LL);
    out[0] = V;
    out[1] = cen[0];
    out[2] = cen[1];
    out[3] = cen[2];
    out[4] = (ra - rc) / (ra + rc);
    out[5] = th;
    out[6] = ra;
    out[7] = rb;
    out[8] = rc;
    out[9] = s7[6];
    for (int q = 0; q < 6; ++q) out[10 + q] = I[q];
    if (aux) {
      aux[0] = V;
      for (int q = 0; q < 6; ++q) aux[1 + q] = s7[q];
      for (int k = 0; k < 3; ++k) {
        aux[7 + k] = e[id[k]];
        for (int d = 0; d < 3; ++d) aux[10 + 3 * k + d] = vec[d][id[k]];
      }
    }
    finite = isfinite(V) && isfinite(out[4]);
    for (int q = 0; q < 6; ++q) finite = finite && isfinite(I[q]);
  }
  return finite;
}

__global__ __launch_bounds__(256) void k_observables(MemDev M, Ctrl *ctrl, const float4 *dx,
                                                     double h, double *obs) {
  __shared__ double red[7][256];
  __shared__ double cen[3];
  const int c = blockIdx.x;
  double out[16];
  const bool finite = capsule_obs(M, c, PosShift{&M, dx, h}, red, cen, out);
  if (threadIdx.x != 0) return;
  const int4 o = M.origin[c];
  out[1] += o.x;
  out[2] += o.y;
  out[3] += o.z;
  for (int q = 0; q < 16; ++q) obs[(size_t)c * 16 + q] = out[q];
  if (!finite) atomicOr(&ctrl->err, ERR_NONFINITE);
}

// dD/dx of capsule c at the stored node positions (Sec. III), by reverse
// differentiation of the observables:
//   D = (r_a - r_c)/(r_a + r_c), r_a^2 = 5/2 (E2 + E3 - E1),
//   r_c^2 = 5/2 (E1 + E2 - E3);
//   dE_k = v_k^T dI v_k for the eigenpairs of I (distinct eigenvalues), so
//   dD/dI = sum_k dD/dE_k v_k v_k^T;
//   I = S / (5 V) with the face sums S = sum_f Q(r_f) (r_f . a_f),
//   Q(r) = |r|^2 1 - r r^T, r_f the face centroid relative to the volume
//   centroid c and a_f = (x2 - x1) x (x3 - x1) / 2 the area normal;
//   V = sum_f x1 . (x2 x x3) / 6 and c = sum_f v_f (x1 + x2 + x3) / (4 V).
// Thread 0 forms the capsule-level adjoints (of S, V and of the centroid's
// numerator, the latter after a block sum of -sum_f dD/dr_f); then every
// node gathers the contributions of its incident faces (deterministic sums)
// and writes FP64 (out64) or FP32 (out32, xyz of a float4) at its internal
// index.  One block per call.
struct FaceAdj {
  double Sb[6];   // dD/dS
  double Vb;      // dD/dV through I and the centroid
  double Pb[3];   // dD/d(sum_f v_f (x1 + x2 + x3) / 4)
};

__device__ __forceinline__ void face_r_adjoint(const double3 A, const double3 B, const double3 C,
                                               const double *cen, const double *Sb, double3 &r,
                                               double3 &an, double3 &rb, double &P) {
  const double3 e1 = make_double3(B.x - A.x, B.y - A.y, B.z - A.z);
  const double3 e2 = make_double3(C.x - A.x, C.y - A.y, C.z - A.z);
  an = make_double3(0.5 * (e1.y * e2.z - e1.z * e2.y), 0.5 * (e1.z * e2.x - e1.x * e2.z),
                    0.5 * (e1.x * e2.y - e1.y * e2.x));
  r = make_double3((A.x + B.x + C.x) / 3.0 - cen[0], (A.y + B.y + C.y) / 3.0 - cen[1],
                   (A.z + B.z + C.z) / 3.0 - cen[2]);
  const double rn = r.x * an.x + r.y * an.y + r.z * an.z;
  // sum_q Sb_q Q_q(r) = r^T K r with K = [[Sb1 + Sb2, -Sb3/2, -Sb4/2], ...]
  const double k00 = Sb[1] + Sb[2], k11 = Sb[0] + Sb[2], k22 = Sb[0] + Sb[1];
  const double k01 = -0.5 * Sb[3], k02 = -0.5 * Sb[4], k12 = -0.5 * Sb[5];
  const double kx = k00 * r.x + k01 * r.y + k02 * r.z;
  const double ky = k01 * r.x + k11 * r.y + k12 * r.z;
  const double kz = k02 * r.x + k12 * r.y + k22 * r.z;
  P = r.x * kx + r.y * ky + r.z * kz;
  rb = make_double3(2.0 * rn * kx + P * an.x, 2.0 * rn * ky + P * an.y, 2.0 * rn * kz + P * an.z);
}

template <typename O>
__device__ void obs_grad_D(const MemDev &M, int c, O out) {
  __shared__ double red[7][256];
  __shared__ double cen[3];
  __shared__ double aux[19];
  __shared__ FaceAdj fa;
  const PosShift pos{&M, nullptr, 0.0};
  double o[16];
  capsule_obs(M, c, pos, red, cen, o, threadIdx.x == 0 ? aux : nullptr);
  if (threadIdx.x == 0) {
    const double V = aux[0];
    const double E1 = aux[7], E2 = aux[8], E3 = aux[9];
    const double ra = sqrt(fmax(2.5 * (E2 + E3 - E1), 0.0));
    const double rc = sqrt(fmax(2.5 * (E1 + E2 - E3), 0.0));
    const double den = (ra + rc) * (ra + rc);
    const double dra = 2.0 * rc / den, drc = -2.0 * ra / den;
    const double ga = ra > 0.0 ? 1.25 / ra : 0.0, gc = rc > 0.0 ? 1.25 / rc : 0.0;
    const double gE[3] = {-dra * ga + drc * gc, dra * ga + drc * gc, dra * ga - drc * gc};
    double Ib[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Ib[i][j] += gE[k] * aux[10 + 3 * k + i] * aux[10 + 3 * k + j];
    // I_q = S_q / (5 V); the off-diagonal I_q sits twice in the matrix
    const double dI[6] = {Ib[0][0], Ib[1][1], Ib[2][2], 2.0 * Ib[0][1], 2.0 * Ib[0][2],
                          2.0 * Ib[1][2]};
    double vb = 0.0;
    for (int q = 0; q < 6; ++q) {
      fa.Sb[q] = dI[q] / (5.0 * V);
      vb -= dI[q] * aux[1 + q] / (5.0 * V * V);
    }
    fa.Vb = vb;
  }
  __syncthreads();
  // dD/dc = -sum_f dD/dr_f
  const int f0 = M.cap_face_off[c], f1 = M.cap_face_off[c + 1];
  double cb[3] = {0.0, 0.0, 0.0};
  for (int j = f0 + threadIdx.x; j < f1; j += blockDim.x) {
    const int4 t = M.tri[j];
    double3 r, an, rb;
    double P;
    face_r_adjoint(pos(t.x), pos(t.y), pos(t.z), cen, fa.Sb, r, an, rb, P);
    cb[0] -= rb.x;
    cb[1] -= rb.y;
    cb[2] -= rb.z;
  }
  block_sum<3>(red, cb);
  if (threadIdx.x == 0) {
    const double V = aux[0];
    // c = Pnum / V: dD/dPnum = cb / V, and V gains -cb . c / V
    for (int d = 0; d < 3; ++d) fa.Pb[d] = cb[d] / V;
    fa.Vb -= (cb[0] * cen[0] + cb[1] * cen[1] + cb[2] * cen[2]) / V;
  }
  __syncthreads();
  const int n0 = M.cap_node_off[c], n1 = M.cap_node_off[c + 1];
  for (int n = n0 + threadIdx.x; n < n1; n += blockDim.x) {
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int e = M.csr_off[n]; e < M.csr_off[n + 1]; ++e) {
      const int ent = M.csr_ent[e];
      const int4 t = M.tri[ent >> 2];
      const int corner = ent & 3;
      const double3 A = pos(t.x), B = pos(t.y), C = pos(t.z);
      double3 r, an, rb;
      double P;
      face_r_adjoint(A, B, C, cen, fa.Sb, r, an, rb, P);
      // the face centroid moves by a third of each corner's motion
      double g[3] = {rb.x / 3.0, rb.y / 3.0, rb.z / 3.0};
      // the area normal a = (B - A) x (C - A) / 2 with adjoint P r:
      // dB = (C - A) x (P r) / 2, dC = (P r) x (B - A) / 2, dA = -(dB + dC)
      const double3 ab = make_double3(P * r.x, P * r.y, P * r.z);
      const double3 e1 = make_double3(B.x - A.x, B.y - A.y, B.z - A.z);
      const double3 e2 = make_double3(C.x - A.x, C.y - A.y, C.z - A.z);
      const double bB[3] = {0.5 * (e2.y * ab.z - e2.z * ab.y), 0.5 * (e2.z * ab.x - e2.x * ab.z),
                            0.5 * (e2.x * ab.y - e2.y * ab.x)};
      const double bC[3] = {0.5 * (ab.y * e1.z - ab.z * e1.y), 0.5 * (ab.z * e1.x - ab.x * e1.z),
                            0.5 * (ab.x * e1.y - ab.y * e1.x)};
      // volume v = A . (B x C) / 6 (adjoint w = Vb + Pb . (A + B + C) / 4)
      // and the centroid numerator v (A + B + C) / 4
      const double vt = (A.x * (B.y * C.z - B.z * C.y) + A.y * (B.z * C.x - B.x * C.z) +
                         A.z * (B.x * C.y - B.y * C.x)) / 6.0;
      const double w = fa.Vb + 0.25 * (fa.Pb[0] * (A.x + B.x + C.x) + fa.Pb[1] * (A.y + B.y + C.y) +
                                       fa.Pb[2] * (A.z + B.z + C.z));
      double cr[3];
      if (corner == 0) {
        cr[0] = B.y * C.z - B.z * C.y; cr[1] = B.z * C.x - B.x * C.z; cr[2] = B.x * C.y - B.y * C.x;
        for (int d = 0; d < 3; ++d) g[d] -= bB[d] + bC[d];
      } else if (corner == 1) {
        cr[0] = C.y * A.z - C.z * A.y; cr[1] = C.z * A.x - C.x * A.z; cr[2] = C.x * A.y - C.y * A.x;
        for (int d = 0; d < 3; ++d) g[d] += bB[d];
      } else {
        cr[0] = A.y * B.z - A.z * B.y; cr[1] = A.z * B.x - A.x * B.z; cr[2] = A.x * B.y - A.y * B.x;
        for (int d = 0; d < 3; ++d) g[d] += bC[d];
      }
      for (int d = 0; d < 3; ++d) g[d] += w * cr[d] / 6.0 + 0.25 * vt * fa.Pb[d];
      gx += g[0];
      gy += g[1];
      gz += g[2];
    }
    out(n, gx, gy, gz);
  }
}

struct GradOut32 {
  float4 *g;
  __device__ void operator()(int n, double x, double y, double z) const {
    g[n] = make_float4((float)x, (float)y, (float)z, 0.0f);
  }
};
// FP64 rows in the caller's node order
struct GradOut64 {
  const int *ext;
  double *g;
  __device__ void operator()(int n, double x, double y, double z) const {
    const int r = ext[n];
    g[3 * (long long)r] = x;
    g[3 * (long long)r + 1] = y;
    g[3 * (long long)r + 2] = z;
  }
};

__global__ __launch_bounds__(256) void k_obs_grad32(MemDev M, int c, float4 *grad) {
  obs_grad_D(M, c, GradOut32{grad});
}
__global__ __launch_bounds__(256) void k_obs_grad64(MemDev M, int c, double *grad) {
  obs_grad_D(M, c, GradOut64{M.ext_id, grad});
}

void launch_obs_grad(const MemDev &M, int c, float4 *grad, hipStream_t s) {
  k_obs_grad32<<<dim3(1), dim3(256), 0, s>>>(M, c, grad);
}

void launch_obs_grad64(const MemDev &M, int c, double *grad, hipStream_t s) {
  k_obs_grad64<<<dim3(1), dim3(256), 0, s>>>(M, c, grad);
}

void launch_observables(const MemDev &M, Ctrl *ctrl, hipStream_t s) {
  if (M.n_caps <= 0) return;
  k_observables<<<dim3(M.n_caps), dim3(256), 0, s>>>(M, ctrl, nullptr, 0.0, M.obs);
}

void launch_observables_shifted(const MemDev &M, Ctrl *ctrl, const float4 *dx, double h,
                                double *obs, hipStream_t s) {
  if (M.n_caps <= 0) return;
  k_observables<<<dim3(M.n_caps), dim3(256), 0, s>>>(M, ctrl, dx, h, obs);
}

// ---- mesh output (FP64, unwrapped lattice coordinates) -----------------------------
// Node n (internal, spatially sorted order) goes to row ext_id[n] (the
// caller's order).
__global__ __launch_bounds__(256) void k_get_mesh(MemDev M, double *xyz, double *F, double *u) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= M.nn) return;
  const int e = M.ext_id[n];
  if (xyz) {
    const float4 p = M.x[n];
    const int4 o = M.origin[M.node_cap[n]];
    xyz[3 * e + 0] = (double)o.x + (double)p.x;
    xyz[3 * e + 1] = (double)o.y + (double)p.y;
    xyz[3 * e + 2] = (double)o.z + (double)p.z;
  }
  if (F) {
    const float4 f = M.F[n];
    F[3 * e + 0] = f.x;
    F[3 * e + 1] = f.y;
    F[3 * e + 2] = f.z;
  }
  if (u) {
    const float4 v = M.u[n];
    u[3 * e + 0] = v.x;
    u[3 * e + 1] = v.y;
    u[3 * e + 2] = v.z;
  }
}

void launch_get_mesh(const MemDev &M, double *xyz, double *F, double *u, hipStream_t s) {
  if (M.nn <= 0) return;
  k_get_mesh<<<dim3((M.nn + 255) / 256), dim3(256), 0, s>>>(M, xyz, F, u);
}

}  // namespace ibm
