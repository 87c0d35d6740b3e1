// Device code of the lattice update shared by the lattice kernels and the
// coupling kernels that carry part of a split lattice update: population
// storage access, the BGK + Guo collision (Sec. II.A), and the row-form
// collide-stream of one x-row segment.  Not part of the public ABI.
#pragma once

#include "common.h"

namespace ibm {


// Population storage access.  FP32: the deviation itself.  FP16: the
// deviation times a per-direction scale.  NT selects non-temporal loads and
// stores (streamed data that will not be reused before it leaves the caches).
typedef float f32x2 __attribute__((ext_vector_type(2)));

template <typename T>
struct Pop;

template <>
struct Pop<float> {
  template <bool NT>
  static __device__ __forceinline__ float ld(const float *p, long long i, float) {
    if (NT) return __builtin_nontemporal_load(p + i);
    return p[i];
  }
  template <bool NT>
  static __device__ __forceinline__ void ld2(const float *p, long long i, float, float &a, float &b) {
    const f32x2 *q = reinterpret_cast<const f32x2 *>(p + i);
    const f32x2 v = NT ? __builtin_nontemporal_load(q) : *q;
    a = v.x;
    b = v.y;
  }
  template <bool NT>
  static __device__ __forceinline__ void st(float *p, long long i, float v, float) {
    if (NT) __builtin_nontemporal_store(v, p + i);
    else p[i] = v;
  }
  template <bool NT>
  static __device__ __forceinline__ void st2(float *p, long long i, float a, float b, float) {
    f32x2 v;
    v.x = a;
    v.y = b;
    f32x2 *q = reinterpret_cast<f32x2 *>(p + i);
    if (NT) __builtin_nontemporal_store(v, q);
    else *q = v;
  }
};

template <>
struct Pop<__half> {
  template <bool NT>
  static __device__ __forceinline__ float ld(const __half *p, long long i, float inv) {
    const unsigned short *q = reinterpret_cast<const unsigned short *>(p) + i;
    const unsigned short r = NT ? __builtin_nontemporal_load(q) : *q;
    return __half2float(__ushort_as_half(r)) * inv;
  }
  template <bool NT>
  static __device__ __forceinline__ void ld2(const __half *p, long long i, float inv, float &a,
                                             float &b) {
    const unsigned int *q = reinterpret_cast<const unsigned int *>(p + i);
    const unsigned int r = NT ? __builtin_nontemporal_load(q) : *q;
    a = __half2float(__ushort_as_half((unsigned short)(r & 0xffffu))) * inv;
    b = __half2float(__ushort_as_half((unsigned short)(r >> 16))) * inv;
  }
  template <bool NT>
  static __device__ __forceinline__ void st(__half *p, long long i, float v, float scale) {
    const unsigned short r = __half_as_ushort(__float2half_rn(v * scale));
    unsigned short *q = reinterpret_cast<unsigned short *>(p) + i;
    if (NT) __builtin_nontemporal_store(r, q);
    else *q = r;
  }
  template <bool NT>
  static __device__ __forceinline__ void st2(__half *p, long long i, float a, float b, float scale) {
    const unsigned int r = (unsigned int)__half_as_ushort(__float2half_rn(a * scale)) |
                           ((unsigned int)__half_as_ushort(__float2half_rn(b * scale)) << 16);
    unsigned int *q = reinterpret_cast<unsigned int *>(p + i);
    if (NT) __builtin_nontemporal_store(r, q);
    else *q = r;
  }
};

// Scalar accessors for the non-hot kernels.
template <typename T>
__device__ __forceinline__ float ld_dev(const T *p, long long idx, float inv_scale) {
  return Pop<T>::template ld<false>(p, idx, inv_scale);
}
template <typename T>
__device__ __forceinline__ void st_dev(T *p, long long idx, float v, float scale) {
  Pop<T>::template st<false>(p, idx, v, scale);
}

// Post-collision deviations of one node.
//   Moments (Eqs. lbmmomenta0/1): rho = 1 + sum d_i, rho u = sum c_i d_i + g/2
//   (sum c_i w_i = 0).  Equilibrium deviation (Eq. equilibrium):
//   feq_i - w_i = w_i (rho - 1) + w_i rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u),
//   or w_i (rho - 1) + 3 w_i rho c.u for the linearised form (Sec. IV.A).
//   Guo term (Eq. latticeforce) and BGK relaxation (Eq. lbequation):
//   d_i' = (1 - 1/tau) d_i + (feq_i - w_i) / tau
//          + (1 - 1/(2 tau)) w_i (3 (c_i - u).g + 9 (c_i.u)(c_i.g)).
// Evaluated as d_i' = (1 - 1/tau) d_i + w_i t(c_i.u, c_i.e) with e = 3 (1 -
// 1/(2 tau)) g and the node scalars of
//   t(p, q) = C0 + a p + b p^2 + q + 3 p q,
//   C0 = (rho - 1 - 3/2 rho u.u) / tau - u.e,  a = 3 rho / tau,
//   b = 9/2 rho / tau (the linearised form: no u.u term, b = 0).
// A pair of opposite directions has (p, q) and (-p, -q), so each pair costs
// the even part S = C0 + p (b p + 3 q) and the odd part A = a p + q once:
// t = S + A and S - A.
constexpr bool odd_even_pairs_opposite() {
  for (int i = 1; i < Q; i += 2)
    if (cx(i + 1) != -cx(i) || cy(i + 1) != -cy(i) || cz(i + 1) != -cz(i) || wgt(i + 1) != wgt(i))
      return false;
  return true;
}
static_assert(odd_even_pairs_opposite(), "directions 2k-1 and 2k must be opposite");

// c_i . (x, y, z) as a signed sum of the nonzero components only (a product
// with a zero component is not folded away under IEEE rules; -0 + v is).
__device__ __forceinline__ float cdot(int i, float x, float y, float z) {
  float r = -0.0f;
  if (cx(i) > 0) r = r + x;
  if (cx(i) < 0) r = r - x;
  if (cy(i) > 0) r = r + y;
  if (cy(i) < 0) r = r - y;
  if (cz(i) > 0) r = r + z;
  if (cz(i) < 0) r = r - z;
  return r;
}

// The moving-wall term of a population that bounces back: 6 w_i (c_i . u_w)
// with the wall moving along x at -uw (bottom, c_z < 0) or +uw (top).
__device__ __forceinline__ float wall_kick(int i, float uw) {
  if (cx(i) == 0) return 0.0f;
  return 6.0f * (float)wgt(i) * (float)(cx(i) * (cz(i) < 0 ? -1 : 1)) * uw;
}

// SCALED: d holds D_i = (f_i - w_i) 16 / w_i, the FP16 storage units, in and
// out.  The moments take w_i / 16 per weight class, and the update becomes
// D_i' = (1 - 1/tau) D_i + 16 t(c_i.u, c_i.e): the factor 16 goes into the node
// scalars, so neither the load nor the store needs a per-direction scale.
template <bool LINEAR, bool FORCE, bool SCALED = false>
__device__ __forceinline__ void collide(float (&d)[Q], float gx, float gy, float gz,
                                        float inv_tau, float guo_pre) {
  // partial sums per weight class: rest, axis (1-6), diagonal (7-18)
  float sa = -0.0f, sd = -0.0f, xa = -0.0f, xd = -0.0f, ya = -0.0f, yd = -0.0f, za = -0.0f,
        zd = -0.0f;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    float &s = i <= 6 ? sa : sd, &jx = i <= 6 ? xa : xd, &jy = i <= 6 ? ya : yd,
          &jz = i <= 6 ? za : zd;
    s = s + d[i];
    if (cx(i) > 0) jx = jx + d[i];
    if (cx(i) < 0) jx = jx - d[i];
    if (cy(i) > 0) jy = jy + d[i];
    if (cy(i) < 0) jy = jy - d[i];
    if (cz(i) > 0) jz = jz + d[i];
    if (cz(i) < 0) jz = jz - d[i];
  }
  constexpr float k0 = SCALED ? (float)(wgt(0) / 16.0) : 1.0f;
  constexpr float ka = SCALED ? (float)(wgt(1) / 16.0) : 1.0f;
  constexpr float kd = SCALED ? (float)(wgt(7) / 16.0) : 1.0f;
  const float drho = k0 * d[0] + ka * sa + kd * sd;
  const float jx = ka * xa + kd * xd, jy = ka * ya + kd * yd, jz = ka * za + kd * zd;
  const float rho = 1.0f + drho;
  const float inv_rho = __builtin_amdgcn_rcpf(rho);  // 1 ulp; rho is near 1
  float ux = jx, uy = jy, uz = jz;
  if (FORCE) {
    ux += 0.5f * gx;
    uy += 0.5f * gy;
    uz += 0.5f * gz;
  }
  ux *= inv_rho;
  uy *= inv_rho;
  uz *= inv_rho;
  constexpr float sc = SCALED ? 16.0f : 1.0f;
  const float om1 = 1.0f - inv_tau;
  const float a = (3.0f * sc) * inv_tau * rho;
  const float b = LINEAR ? 0.0f : 1.5f * a;
  float C0 = LINEAR ? drho * (sc * inv_tau)
                    : (drho - 1.5f * rho * (ux * ux + uy * uy + uz * uz)) * (sc * inv_tau);
  float ex = 0.0f, ey = 0.0f, ez = 0.0f;
  if (FORCE) {
    const float e = (3.0f * sc) * guo_pre;
    ex = e * gx;
    ey = e * gy;
    ez = e * gz;
    C0 -= ux * ex + uy * ey + uz * ez;
  }
  if (SCALED) d[0] = om1 * d[0] + C0;
  else d[0] = om1 * d[0] + (float)wgt(0) * C0;
#pragma unroll
  for (int i = 1; i < Q; i += 2) {
    const float p = cdot(i, ux, uy, uz);
    const float q = FORCE ? cdot(i, ex, ey, ez) : 0.0f;
    const float S = C0 + p * (b * p + 3.0f * q);
    const float A = a * p + q;
    if (SCALED) {
      d[i] = om1 * d[i] + (S + A);
      d[i + 1] = om1 * d[i + 1] + (S - A);
    } else {
      const float w = (float)wgt(i);
      d[i] = om1 * d[i] + w * (S + A);
      d[i + 1] = om1 * d[i + 1] + w * (S - A);
    }
  }
}

// The wall term in FP16 storage units: 6 w_i (c_i . u_w) 16 / w_i.
__device__ __forceinline__ float wall_kick_scaled(int i, float uw) {
  if (cx(i) == 0) return 0.0f;
  return 96.0f * (float)(cx(i) * (cz(i) < 0 ? -1 : 1)) * uw;
}

// FP16 storage, in storage units D_i = (f_i - w_i) 16 / w_i: rounding the 18
// moving post-collision values of a node to FP16 changes the mass the node
// passes on by sum_i (w_i / 16) e_i, e_i = v_i - fp16(v_i) for the value v_i
// that is stored (D_i, less the wall term where the value bounces back from a
// wall: KICK).  The rest population stays at the node; adding
// sum_i (w_i / w_0) e_i to D_0 makes the node's stored values carry its FP32
// mass, up to the rounding of D_0 itself (IBM_OPT_FP16_MASS).  The rounding
// is the stores' own: to nearest even.
template <bool KICK>
__device__ __forceinline__ void fp16_mass_fix(const LatDev &L, int z, float (&d)[4][Q]) {
  float r[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int zt = z + cz(i);
    const bool wall = KICK && cz(i) != 0 && (zt < 0 || zt >= L.nz);
    const float kick = wall ? wall_kick_scaled(i, L.uw) : 0.0f;
    const float wr = (float)(wgt(i) / wgt(0));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float v = d[k][i] - kick;
      r[k] += wr * (v - (float)(_Float16)v);
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) d[k][0] += r[k];
}

// 32-bit form of prow / nx (the group-row index of an x row): row + (Q - 1) G
// (row / G).  Valid while the padded row count times Q is below 2^32, which
// the launchers of its users check.
__host__ __device__ __forceinline__ unsigned grow32(const LatDev &L, unsigned row) {
  return row + (((row >> L.gsh) * (unsigned)(Q - 1)) << L.gsh);
}
// Element offset of (row, x) within population 0 of its group.
__host__ __device__ __forceinline__ unsigned long long rowoff(const LatDev &L, unsigned row, int x) {
  return (unsigned long long)grow32(L, row) * (unsigned)L.nxs + (unsigned)x;
}

// Row-vector form of the same update for rows that fit one wavefront: each
// thread owns 4 consecutive x nodes of the padded row, tpr = nxs / 4 lanes of
// one wavefront hold one whole row and a wavefront holds rpw = 64 / tpr rows
// (lanes beyond rpw tpr idle), so every population is loaded and stored as one
// aligned vector (16 bytes in FP32, 8 in FP16).  The +-x streaming shift moves
// one value per row segment to the neighbouring lane with a lane shuffle; the
// row's ends wrap into each other (the periodic boundary along x), at
// position e = nx - 1 - 4 (tpr - 1) of the last segment when the row is
// padded (values at x >= nx are computed and written into the padding only).
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Pop4;

// NT (default): non-temporal accesses, for populations streamed once per
// step; false: ordinary cached accesses (the row form's stores on lattices
// whose new population buffer largely stays in the last-level cache until
// the next step reads it).
template <>
struct Pop4<float> {
  template <bool NT = true>
  static __device__ __forceinline__ void ld(const float *p, long long i, float, float (&v)[4]) {
    const f32x4 *q = reinterpret_cast<const f32x4 *>(p + i);
    const f32x4 r = NT ? __builtin_nontemporal_load(q) : *q;
    v[0] = r.x;
    v[1] = r.y;
    v[2] = r.z;
    v[3] = r.w;
  }
  template <bool NT = true>
  static __device__ __forceinline__ void st(float *p, long long i, float a, float b, float c,
                                            float d, float) {
    f32x4 r;
    r.x = a;
    r.y = b;
    r.z = c;
    r.w = d;
    f32x4 *q = reinterpret_cast<f32x4 *>(p + i);
    if (NT) __builtin_nontemporal_store(r, q);
    else *q = r;
  }
};

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

template <>
struct Pop4<__half> {
  static __device__ __forceinline__ float h(unsigned int bits, float inv) {
    return __half2float(__ushort_as_half((unsigned short)bits)) * inv;
  }
  static __device__ __forceinline__ unsigned int q(float v, float scale) {
    return (unsigned int)__half_as_ushort(__float2half_rn(v * scale));
  }
  template <bool NT = true>
  static __device__ __forceinline__ void ld(const __half *p, long long i, float inv, float (&v)[4]) {
    const u32x2 *a = reinterpret_cast<const u32x2 *>(p + i);
    const u32x2 r = NT ? __builtin_nontemporal_load(a) : *a;
    v[0] = h(r.x & 0xffffu, inv);
    v[1] = h(r.x >> 16, inv);
    v[2] = h(r.y & 0xffffu, inv);
    v[3] = h(r.y >> 16, inv);
  }
  // two values per conversion: packed float -> half, rounded to nearest even
  // (one v_cvt_pk_f16_f32 instead of two conversions and a pack)
  static __device__ __forceinline__ unsigned int pk(float a, float b) {
    const f32x2 v = {a, b};
    return __builtin_bit_cast(unsigned int, __builtin_convertvector(v, f16x2));
  }
  template <bool NT = true>
  static __device__ __forceinline__ void st(__half *p, long long i, float a, float b, float c,
                                            float d, float scale) {
    u32x2 r;
    r.x = pk(a * scale, b * scale);
    r.y = pk(c * scale, d * scale);
    u32x2 *q = reinterpret_cast<u32x2 *>(p + i);
    if (NT) __builtin_nontemporal_store(r, q);
    else *q = r;
  }
};

// Streaming patterns of the row form (template argument AA):
//   0  two buffers: read f(t) at the node from buffer src, push the
//      post-collision values to the neighbours in buffer src ^ 1;
//   1  AA, even step, one buffer (buffer 0): read the node's own values,
//      write the post-collision values back to the same node in the opposite
//      slot, A[opp(i)][x] = f*_i(x) (no streaming);
//   2  AA, odd step, buffer 0: the post-stream values of the even step are
//      gathered, f_i(x) = A[opp(i)][x - c_i] (or, arriving from a wall,
//      A[i][x] less the wall term of the opposite direction), collided and
//      pushed, A[i][x + c_i] = f**_i(x) (at a wall: back into the node's
//      opposite slot with the wall term), which leaves post-stream values at
//      their own nodes again.
// In the AA steps every location a node reads is written only by that node,
// after its reads (all 19 values are loaded before any store), so one buffer
// suffices.  AA needs rows that are a multiple of 4 long (no padding).

// x row `row`, segment t (lane `lane` of its wavefront).  All lanes of the
// wavefront call this together (the shuffles need every lane); `live` is
// false for idle lanes and rows beyond the lattice.  PAD: nx is not a
// multiple of 4.
template <typename T, bool LINEAR, bool FORCE, bool PAD, bool NT, int AA = 0>
__device__ __forceinline__ void collide_stream_rowseg_a(const LatDev &L, int src, int par, int row,
                                                        int t, int lane, bool live);

// cached: this wavefront stores with cached writes (uniform across it)
template <typename T, bool LINEAR, bool FORCE, bool PAD, int AA = 0>
__device__ __forceinline__ void collide_stream_rowseg(const LatDev &L, int src, int par, int row,
                                                      int t, int lane, bool live, bool cached) {
  if (cached)
    collide_stream_rowseg_a<T, LINEAR, FORCE, PAD, false, AA>(L, src, par, row, t, lane, live);
  else
    collide_stream_rowseg_a<T, LINEAR, FORCE, PAD, true, AA>(L, src, par, row, t, lane, live);
}

// NT: non-temporal population stores (see Pop4); the loads are always
// non-temporal
template <typename T, bool LINEAR, bool FORCE, bool PAD, bool NT, int AA>
__device__ __forceinline__ void collide_stream_rowseg_a(const LatDev &L, int src, int par, int row,
                                                        int t, int lane, bool live) {
  static_assert(!(AA && PAD), "the AA pattern needs rows that are a multiple of 4 long");
  // FP16 values are used in their storage units (collide<..., SCALED>)
  constexpr bool SC = sizeof(T) == 2;
  const int tpr = L.tpr, last = tpr - 1;
  const int y = live ? row % L.ny : 0;
  const int z = live ? row / L.ny : 0;
  const int x0 = t * 4;
  // nodes of this segment inside the row, and the slot of x = nx - 1 in the
  // last segment
  const int nval = PAD ? min(4, L.nx - x0) : 4;
  const int e = PAD ? L.nx - 1 - 4 * last : 3;
  const long long n0 = ((long long)z * L.ny + y) * L.nx + x0;
  const unsigned row0 = (unsigned)(z * L.ny + y);
  const unsigned long long off0 = rowoff(L, row0, x0);
  T *__restrict__ fd = static_cast<T *>(L.f[AA ? 0 : (src ^ 1)]);
  // lanes holding the left and right neighbours of this segment in the row
  const int row_lane0 = lane - t;
  const int left = live ? row_lane0 + (t == 0 ? last : t - 1) : lane;
  const int right = live ? row_lane0 + (t == last ? 0 : t + 1) : lane;

  float d[4][Q];
  if constexpr (AA == 2) {
    // gather the even step's post-collision values from the neighbours; the
    // +-x shift by lane shuffles (every lane takes part)
    const T *fa = static_cast<const T *>(L.f[0]);
    const int ysm = (y == 0) ? L.ny - 1 : y - 1, ysp = (y == L.ny - 1) ? 0 : y + 1;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      const int zs = z - cz(i);
      const bool wall = cz(i) != 0 && (zs < 0 || zs >= L.nz);
      if (live) {
        if (wall) {
          Pop4<T>::template ld<true>(fa + L.pst[i], off0, 1.0f, v);
          const float kick = SC ? wall_kick_scaled(opp(i), L.uw) : wall_kick(opp(i), L.uw);
#pragma unroll
          for (int k = 0; k < 4; ++k) v[k] -= kick;
        } else {
          const int ys = cy(i) > 0 ? ysm : (cy(i) < 0 ? ysp : y);
          Pop4<T>::template ld<true>(fa + L.pst[opp(i)], rowoff(L, (unsigned)(zs * L.ny + ys), x0), 1.0f,
                                     v);
        }
      }
      // node x takes the value of x - c_x: from the left neighbour's last
      // node for c_x > 0, the right neighbour's first for c_x < 0
      if (cx(i) > 0) {
        const float in = __shfl(v[3], left);
        if (!wall) {
          v[3] = v[2];
          v[2] = v[1];
          v[1] = v[0];
          v[0] = in;
        }
      } else if (cx(i) < 0) {
        const float in = __shfl(v[0], right);
        if (!wall) {
          v[0] = v[1];
          v[1] = v[2];
          v[2] = v[3];
          v[3] = in;
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) d[k][i] = v[k];
    }
  }
  if (live) {
    if constexpr (AA != 2) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        float v[4];
        Pop4<T>::template ld<true>(static_cast<const T *>(L.f[AA ? 0 : src]) + L.pst[i], off0, 1.0f, v);
#pragma unroll
        for (int k = 0; k < 4; ++k) d[k][i] = v[k];
      }
    }
    float g[4][3];
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k][0] = g[k][1] = g[k][2] = 0.0f;
    if (FORCE) {
      // the force density is unpadded, three components per node (gix): the
      // segment's 12 values are three aligned vectors when nx is a multiple
      // of 4
      const int step = L.ctrl->step;
      const int tile = tile_of(L, x0, y, z);
      if (L.stamp[par][tile] == step) {
        if (PAD) {
#pragma unroll
          for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c)
              if (k < nval) g[k][c] = L.g[par][gix(n0 + k, c)];
        } else {
          float v[12];
#pragma unroll
          for (int h = 0; h < 3; ++h) {
            float w4[4];
            Pop4<float>::ld(L.g[par], gix(n0, 0) + 4 * h, 1.0f, w4);
#pragma unroll
            for (int k = 0; k < 4; ++k) v[4 * h + k] = w4[k];
          }
#pragma unroll
          for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) g[k][c] = v[3 * k + c];
        }
      }
      if (L.stamp[par ^ 1][tile] == step - 1) {
        if (PAD) {
#pragma unroll
          for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c)
              if (k < nval) L.g[par ^ 1][gix(n0 + k, c)] = 0.0f;
        } else {
#pragma unroll
          for (int h = 0; h < 3; ++h)
            Pop4<float>::st(L.g[par ^ 1], gix(n0, 0) + 4 * h, 0.0f, 0.0f, 0.0f, 0.0f, 1.0f);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      collide<LINEAR, FORCE, SC>(d[k], g[k][0], g[k][1], g[k][2], L.inv_tau, L.guo_pre);
    if constexpr (SC) {
      if (L.mass_fix) fp16_mass_fix<AA != 1>(L, z, d);
    }
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
      for (int k = 0; k < 4; ++k) d[k][i] = 0.0f;
  }

  if constexpr (AA == 1) {
    // the even step: post-collision values to the node's own opposite slots
    if (live) {
#pragma unroll
      for (int i = 0; i < Q; ++i)
        Pop4<T>::template st<NT>(fd + L.pst[opp(i)], off0, d[0][i], d[1][i], d[2][i], d[3][i], 1.0f);
    }
    return;
  }
  const int ym = (y == 0) ? L.ny - 1 : y - 1;
  const int yp = (y == L.ny - 1) ? 0 : y + 1;
  const bool wrap = PAD && t == last;  // this segment holds x = nx - 1 at slot e
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    // every lane takes part in the shuffles, live or not
    float in = 0.0f;
    if (cx(i) > 0) {
      // the last segment hands x = nx - 1 on to x = 0 of the row
      float v = d[3][i];
      if (wrap) v = e == 0 ? d[0][i] : (e == 1 ? d[1][i] : (e == 2 ? d[2][i] : d[3][i]));
      in = __shfl(v, left);
    }
    if (cx(i) < 0) in = __shfl(d[0][i], right);
    if (!live) continue;
    const int zt = z + cz(i);
    if (cz(i) != 0 && (zt < 0 || zt >= L.nz)) {
      const float kick = SC ? wall_kick_scaled(i, L.uw) : wall_kick(i, L.uw);
      Pop4<T>::template st<NT>(fd + L.pst[opp(i)], off0, d[0][i] - kick, d[1][i] - kick,
                               d[2][i] - kick, d[3][i] - kick, 1.0f);
    } else {
      const int yt = cy(i) > 0 ? yp : (cy(i) < 0 ? ym : y);
      T *base = fd + L.pst[i];
      const unsigned long long at = rowoff(L, (unsigned)(zt * L.ny + yt), x0);
      if (cx(i) > 0) {
        Pop4<T>::template st<NT>(base, at, in, d[0][i], d[1][i], d[2][i], 1.0f);
      } else if (cx(i) < 0) {
        // slot k takes x0 + k + 1; in the last segment x = nx - 1 (slot e)
        // takes x = 0 of the row (`in`), slots beyond e are padding
        float o0 = d[1][i], o1 = d[2][i], o2 = d[3][i];
        if (wrap) {
          o0 = e == 0 ? in : o0;
          o1 = e <= 1 ? in : o1;
          o2 = e <= 2 ? in : o2;
        }
        Pop4<T>::template st<NT>(base, at, o0, o1, o2, in, 1.0f);
      } else {
        Pop4<T>::template st<NT>(base, at, d[0][i], d[1][i], d[2][i], d[3][i], 1.0f);
      }
    }
  }
}

}  // namespace ibm
