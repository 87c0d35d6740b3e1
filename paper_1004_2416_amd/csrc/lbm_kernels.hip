// Lattice kernels: fused D3Q19 BGK collision with Guo forcing, streaming and
// moving-wall bounce-back (Sec. II.A), equilibrium initialisation, and the
// FP64 field I/O of the public interface.
//
// Storage: populations as deviations d_i = f_i - w_i from the lattice weights
// in the row-group layout of pidx (common.h), in FP32 or in FP16 scaled per
// direction.  Two buffers alternate: the kernel reads f(t) at the node itself
// (aligned loads) and pushes the post-collision values to the neighbours of
// buffer t+1, so both buffers always hold post-streaming populations at their
// own nodes.  A thread block covers whole x rows, so every cache line of the
// destination is written by one block.
#include "common.h"
#include "launch.h"
#include "lbm_device.h"

#include <hip/hip_ext.h>

namespace ibm {

// One lattice update of VEC consecutive x nodes (x0 .. x0 + VEC - 1) of buffer
// `src`, pushed into buffer src ^ 1: streaming to x + c_i, periodic in x and y;
// populations leaving through a wall return to their node reversed, with
// -2 w_i rho_w (c_i . u_wall) / c_s^2, rho_w = 1 (bounce-back for moving
// walls).  VEC = 2 needs an even nx (vector accesses stay aligned).
template <typename T, bool LINEAR, bool FORCE, int VEC, bool NT>
__device__ __forceinline__ void collide_stream_nodes(const LatDev &L, int src, int par, int x0,
                                                     int y, int z) {
  const long long nxl = L.nx;
  const long long plane = nxl * L.ny;
  const long long n0 = (long long)z * plane + (long long)y * nxl + x0;
  const long long row0 = (long long)z * L.ny + y;
  const T *__restrict__ fs = static_cast<const T *>(L.f[src]);
  T *__restrict__ fd = static_cast<T *>(L.f[src ^ 1]);

  float d[VEC][Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float inv = L.h_inv[i];
    const long long at = pidx_c(L, i, row0, x0);
    if constexpr (VEC == 2) Pop<T>::template ld2<NT>(fs, at, inv, d[0][i], d[1][i]);
    else d[0][i] = Pop<T>::template ld<NT>(fs, at, inv);
  }

  float g[VEC][3];
#pragma unroll
  for (int v = 0; v < VEC; ++v) g[v][0] = g[v][1] = g[v][2] = 0.0f;
  if (FORCE) {
    // one tile holds all VEC nodes (TILE_X is a multiple of VEC)
    const int t = L.ctrl->step;
    const int tile = tile_of(L, x0, y, z);
    if (L.stamp[par][tile] == t) {
      const float *gp = L.g[par];
#pragma unroll
      for (int v = 0; v < VEC; ++v)
#pragma unroll
        for (int c = 0; c < 3; ++c) g[v][c] = gp[gix(n0 + v, c)];
    }
    // The other field was spread one step ago and has been interpolated
    // from; clear it where it was touched so the next spreading starts at 0.
    if (L.stamp[par ^ 1][tile] == t - 1) {
      float *go = L.g[par ^ 1];
#pragma unroll
      for (int v = 0; v < VEC; ++v)
#pragma unroll
        for (int c = 0; c < 3; ++c) go[gix(n0 + v, c)] = 0.0f;
    }
  }
#pragma unroll
  for (int v = 0; v < VEC; ++v)
    collide<LINEAR, FORCE>(d[v], g[v][0], g[v][1], g[v][2], L.inv_tau, L.guo_pre);

  const int ym = (y == 0) ? L.ny - 1 : y - 1;
  const int yp = (y == L.ny - 1) ? 0 : y + 1;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int zt = z + cz(i);
    if (cz(i) != 0 && (zt < 0 || zt >= L.nz)) {
      const float kick = wall_kick(i, L.uw);
      const long long at = pidx_c(L, opp(i), row0, x0);
      if constexpr (VEC == 2)
        Pop<T>::template st2<NT>(fd, at, d[0][i] - kick, d[1][i] - kick, L.h_scale[opp(i)]);
      else Pop<T>::template st<NT>(fd, at, d[0][i] - kick, L.h_scale[opp(i)]);
    } else {
      const int yt = cy(i) > 0 ? yp : (cy(i) < 0 ? ym : y);
      const long long row = pidx_c(L, i, (long long)zt * L.ny + yt, 0);
      if (cx(i) == 0) {
        if constexpr (VEC == 2) Pop<T>::template st2<NT>(fd, row + x0, d[0][i], d[1][i], L.h_scale[i]);
        else Pop<T>::template st<NT>(fd, row + x0, d[0][i], L.h_scale[i]);
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          int xt = x0 + v + cx(i);
          xt = xt < 0 ? xt + L.nx : (xt >= L.nx ? xt - L.nx : xt);
          Pop<T>::template st<NT>(fd, row + xt, d[v][i], L.h_scale[i]);
        }
      }
    }
  }
}

template <typename T, bool LINEAR, bool FORCE, int VEC, bool NT>
__global__ __launch_bounds__(256) void k_collide_stream(LatDev L, int src, int par, int z0) {
  const int x0 = (blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = z0 + (int)blockIdx.z;
  if (x0 >= L.nx || y >= L.ny) return;
  collide_stream_nodes<T, LINEAR, FORCE, VEC, NT>(L, src, par, x0, y, z);
}

// The rows of set rs, rpw consecutive ones per wavefront.  AA: the
// streaming pattern (collide_stream_rowseg_a).
template <typename T, bool LINEAR, bool FORCE, bool PAD, int AA = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_collide_stream_rows(
    LatDev L, int src, int par, RowSet rs) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * (int)blockDim.x + (int)threadIdx.x) >> 6;
  const int r = lane / L.tpr;  // row within the wavefront
  const int t = lane - r * L.tpr;
  const int k = wave * L.rpw + r;
  const bool live = r < L.rpw && k < rs.n0 + rs.n1;
  // a single lattice stores all rows or none with cached writes
  collide_stream_rowseg<T, LINEAR, FORCE, PAD, AA>(L, src, par, live ? rowset_row(rs, L, k) : 0, t,
                                                   lane, live, L.cached_rows != 0);
}

// Row kernels index x rows with grow32: the padded row count times Q must stay
// below 2^32.
static bool rows_fit_32bit(const LatDev &L) {
  const long long G = 1LL << L.gsh;
  const long long rows = ((long long)L.ny * L.nz + G - 1) / G * G;
  return rows * Q < (1LL << 32);
}

// Launch k on (g, b); with a timer, through hipExtLaunchKernel so that the
// timer's events take this dispatch's own start and end timestamps.
template <typename K, typename... A>
static void launch_k(K k, dim3 g, dim3 b, hipStream_t s, const DispatchTimer *t, A... a) {
  if (t) hipExtLaunchKernelGGL(k, g, b, 0, s, t->start, t->stop, 0, a...);
  else hipLaunchKernelGGL(k, g, b, 0, s, a...);
}

template <typename T, bool PAD>
static void launch_cs_rows_p(const LatDev &L, int src, int par, bool force, bool linear, dim3 g,
                             dim3 b, const RowSet &rs, hipStream_t s, const DispatchTimer *t) {
  if (force) {
    if (linear) launch_k(k_collide_stream_rows<T, true, true, PAD>, g, b, s, t, L, src, par, rs);
    else launch_k(k_collide_stream_rows<T, false, true, PAD>, g, b, s, t, L, src, par, rs);
  } else {
    if (linear) launch_k(k_collide_stream_rows<T, true, false, PAD>, g, b, s, t, L, src, par, rs);
    else launch_k(k_collide_stream_rows<T, false, false, PAD>, g, b, s, t, L, src, par, rs);
  }
}

// The AA pattern (L.aa; rows a multiple of 4 long): the even step for src =
// 0, the odd step for src = 1 (the step count's parity), both in buffer 0.
template <typename T, int AA>
static void launch_cs_rows_aa(const LatDev &L, int par, bool force, bool linear, dim3 g, dim3 b,
                              const RowSet &rs, hipStream_t s, const DispatchTimer *t) {
  if (force) {
    if (linear) launch_k(k_collide_stream_rows<T, true, true, false, AA>, g, b, s, t, L, 0, par, rs);
    else launch_k(k_collide_stream_rows<T, false, true, false, AA>, g, b, s, t, L, 0, par, rs);
  } else {
    if (linear) launch_k(k_collide_stream_rows<T, true, false, false, AA>, g, b, s, t, L, 0, par, rs);
    else launch_k(k_collide_stream_rows<T, false, false, false, AA>, g, b, s, t, L, 0, par, rs);
  }
}

// wpb: wavefronts per block (1, 2 or 4)
template <typename T>
static bool launch_cs_rows(const LatDev &L, int src, int par, bool force, bool linear,
                           const RowSet &rs, hipStream_t s, const DispatchTimer *t = nullptr,
                           int wpb = 4) {
  if (L.tpr <= 0) return false;
  const long long waves = ((long long)rs.n0 + rs.n1 + L.rpw - 1) / L.rpw;
  if (waves <= 0) return true;
  const dim3 g((unsigned)((waves + wpb - 1) / wpb)), b((unsigned)(64 * wpb));
  if (L.aa) {
    if (src) launch_cs_rows_aa<T, 2>(L, par, force, linear, g, b, rs, s, t);
    else launch_cs_rows_aa<T, 1>(L, par, force, linear, g, b, rs, s, t);
  } else if (L.nx % 4) {
    launch_cs_rows_p<T, true>(L, src, par, force, linear, g, b, rs, s, t);
  } else {
    launch_cs_rows_p<T, false>(L, src, par, force, linear, g, b, rs, s, t);
  }
  return true;
}

// Block shape: whole x rows (up to `threads` nodes / VEC threads), stacked in y.
static dim3 lattice_block(const LatDev &L, int vec = 1, int threads = 256) {
  const int cols = (L.nx + vec - 1) / vec;
  int bx = ((cols + 31) / 32) * 32;
  if (bx > threads) bx = threads;
  int by = threads / bx;
  if (by < 1) by = 1;
  return dim3(bx, by, 1);
}

static dim3 lattice_grid(const LatDev &L, dim3 b, int vec = 1) {
  const int cols = (L.nx + vec - 1) / vec;
  return dim3((cols + b.x - 1) / b.x, (L.ny + b.y - 1) / b.y, L.nz);
}

template <typename T, int VEC, bool NT>
static void launch_cs_v(const LatDev &L, int src, int par, bool force, bool linear,
                        int threads, int z0, int z1, hipStream_t s, const DispatchTimer *t) {
  dim3 b = lattice_block(L, VEC, threads), g = lattice_grid(L, b, VEC);
  g.z = (unsigned)(z1 - z0);
  if (force) {
    if (linear) launch_k(k_collide_stream<T, true, true, VEC, NT>, g, b, s, t, L, src, par, z0);
    else launch_k(k_collide_stream<T, false, true, VEC, NT>, g, b, s, t, L, src, par, z0);
  } else {
    if (linear) launch_k(k_collide_stream<T, true, false, VEC, NT>, g, b, s, t, L, src, par, z0);
    else launch_k(k_collide_stream<T, false, false, VEC, NT>, g, b, s, t, L, src, par, z0);
  }
}

template <typename T>
static void launch_cs_t(const LatDev &L, int src, int par, bool force, bool linear,
                        int variant, int z0, int z1, hipStream_t s, const DispatchTimer *t) {
  // variant bits: 16 = row-vector kernel (four nodes per thread, whole rows
  // per wavefront) where a padded row has at most 256 values, 64 = row form
  // in 128-thread blocks, 128 = in 64-thread blocks; else the per-node kernel
  // with 1 = two nodes per thread, 2 = non-temporal accesses, 4 = 128-thread
  // blocks (256 otherwise)
  const RowSet rs{z0 * L.ny, (z1 - z0) * L.ny, 0, 0, 1, 0};
  const int wpb = (variant & 128) ? 1 : ((variant & 64) ? 2 : 4);
  // the AA pattern and the FP16 mass correction exist in the row form only
  // (they are allowed only there)
  if ((variant & 16 || L.aa || L.mass_fix) && launch_cs_rows<T>(L, src, par, force, linear, rs, s, t, wpb))
    return;
  const bool vec2 = (variant & 1) && (L.nx % 2 == 0);
  const bool nt = (variant & 2) != 0;
  const int threads = (variant & 4) ? 128 : 256;
  if (vec2) {
    if (nt) launch_cs_v<T, 2, true>(L, src, par, force, linear, threads, z0, z1, s, t);
    else launch_cs_v<T, 2, false>(L, src, par, force, linear, threads, z0, z1, s, t);
  } else {
    if (nt) launch_cs_v<T, 1, true>(L, src, par, force, linear, threads, z0, z1, s, t);
    else launch_cs_v<T, 1, false>(L, src, par, force, linear, threads, z0, z1, s, t);
  }
}

bool launch_collide_stream_rows(const LatDev &L, int fp16, int src, int par, bool force,
                                bool linear, const RowSet &rs, hipStream_t s) {
  if (fp16) return launch_cs_rows<__half>(L, src, par, force, linear, rs, s);
  return launch_cs_rows<float>(L, src, par, force, linear, rs, s);
}

void launch_collide_stream(const LatDev &L, int fp16, int src, int par, bool force,
                           bool linear, int variant, hipStream_t s, int z0, int z1,
                           const DispatchTimer *timer) {
  if (z1 < 0) z1 = L.nz;
  if (z0 < 0) z0 = 0;
  if (z1 > L.nz) z1 = L.nz;
  if (z0 >= z1) return;
  if (fp16) launch_cs_t<__half>(L, src, par, force, linear, variant, z0, z1, s, timer);
  else launch_cs_t<float>(L, src, par, force, linear, variant, z0, z1, s, timer);
}

// ---- initialisation: f = feq(rho = 1, u = (uw (2 z + 1 - nz) / nz, 0, 0)) ----
template <typename T>
__global__ __launch_bounds__(256) void k_init_equilibrium(LatDev L, int dst, double uw) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= L.nx || y >= L.ny) return;
  const long long row = (long long)z * L.ny + y;
  const double ux = uw * (2.0 * z + 1.0 - L.nz) / L.nz;
  T *f = static_cast<T *>(L.f[dst]);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double cu = cx(i) * ux;
    const double d = wgt(i) * (3.0 * cu + 4.5 * cu * cu - 1.5 * ux * ux);
    st_dev<T>(f, pidx(L, i, row, x), (float)d, L.h_scale[i]);
  }
}

void launch_init_equilibrium(const LatDev &L, int fp16, int dst, double uw, hipStream_t s) {
  dim3 b = lattice_block(L), g = lattice_grid(L, b);
  if (fp16) k_init_equilibrium<__half><<<g, b, 0, s>>>(L, dst, uw);
  else k_init_equilibrium<float><<<g, b, 0, s>>>(L, dst, uw);
}

// ---- FP64 field I/O ----------------------------------------------------------
// The deviation f_i - w_i a stored value stands for, converted exactly: FP32
// values as they are, FP16 values divided by their scale 16 / w_i (48, 288 or
// 576, exact in FP32) in FP64.
template <typename T>
__device__ __forceinline__ double stored_deviation(const T *f, long long idx, float scale);
template <>
__device__ __forceinline__ double stored_deviation<float>(const float *f, long long idx, float) {
  return (double)f[idx];
}
template <>
__device__ __forceinline__ double stored_deviation<__half>(const __half *f, long long idx,
                                                           float scale) {
  return (double)__half2float(f[idx]) / (double)scale;
}


// The post-stream deviation f_i - w_i at node (x, y, z) of population state
// `state`, converted exactly: 0 or 1, buffer 0 or 1; 2, the AA pattern after
// an even step (the value leaving the source node in the opposite slot of
// buffer 0, or, coming back from a wall, the node's own slot i less the wall
// term of the opposite direction; see collide_stream_rowseg_a).
template <typename T>
__device__ __forceinline__ double stored_post(const LatDev &L, int state, int i, int x, int y,
                                              int z) {
  if (state < 2)
    return stored_deviation<T>(static_cast<const T *>(L.f[state]),
                               pidx(L, i, (long long)z * L.ny + y, x), L.h_scale[i]);
  const T *f = static_cast<const T *>(L.f[0]);
  const int zs = z - cz(i);
  if (cz(i) != 0 && (zs < 0 || zs >= L.nz))
    return stored_deviation<T>(f, pidx(L, i, (long long)z * L.ny + y, x), L.h_scale[i]) -
           (double)wall_kick(opp(i), L.uw);
  const int xs = x - cx(i) < 0 ? L.nx - 1 : (x - cx(i) >= L.nx ? 0 : x - cx(i));
  const int ys = y - cy(i) < 0 ? L.ny - 1 : (y - cy(i) >= L.ny ? 0 : y - cy(i));
  return stored_deviation<T>(f, pidx(L, opp(i), (long long)zs * L.ny + ys, xs), L.h_scale[i]);
}

// what: 0 populations, 1 density, 2 velocity, 3 force density.  gpar: the
// field of the last step (its tiles stamped with that step), or -1 for none.
template <typename T>
__global__ __launch_bounds__(256) void k_get_field(LatDev L, int src, int gpar, int what,
                                                   double *out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= L.nx || y >= L.ny) return;
  const long long N = (long long)L.nx * L.ny * L.nz;
  const long long n = ((long long)z * L.ny + y) * L.nx + x;
  double gx = 0.0, gy = 0.0, gz = 0.0;
  if (gpar >= 0 && L.stamp[gpar][tile_of(L, x, y, z)] == L.ctrl->step - 1) {
    gx = L.g[gpar][gix(n, 0)];
    gy = L.g[gpar][gix(n, 1)];
    gz = L.g[gpar][gix(n, 2)];
  }
  if (what == 3) {
    out[n] = gx;
    out[N + n] = gy;
    out[2 * N + n] = gz;
    return;
  }
  double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double d = stored_post<T>(L, src, i, x, y, z);
    if (what == 0) out[i * N + n] = wgt(i) + d;
    drho += d;
    jx += cx(i) * d;
    jy += cy(i) * d;
    jz += cz(i) * d;
  }
  if (what == 1) out[n] = 1.0 + drho;
  if (what == 2) {
    const double rho = 1.0 + drho;
    out[n] = (jx + 0.5 * gx) / rho;
    out[N + n] = (jy + 0.5 * gy) / rho;
    out[2 * N + n] = (jz + 0.5 * gz) / rho;
  }
}

void launch_get_field(const LatDev &L, int fp16, int src, int gpar, int what, double *out,
                      hipStream_t s) {
  dim3 b = lattice_block(L), g = lattice_grid(L, b);
  if (fp16) k_get_field<__half><<<g, b, 0, s>>>(L, src, gpar, what, out);
  else k_get_field<float><<<g, b, 0, s>>>(L, src, gpar, what, out);
}

template <typename T>
__global__ __launch_bounds__(256) void k_set_pops(LatDev L, int dst, const double *in) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= L.nx || y >= L.ny) return;
  const long long N = (long long)L.nx * L.ny * L.nz;
  const long long n = ((long long)z * L.ny + y) * L.nx + x;
  T *f = static_cast<T *>(L.f[dst]);
#pragma unroll
  for (int i = 0; i < Q; ++i)
    st_dev<T>(f, pidx(L, i, (long long)z * L.ny + y, x), (float)(in[i * N + n] - wgt(i)),
              L.h_scale[i]);
}

void launch_set_pops(const LatDev &L, int fp16, int dst, const double *in, hipStream_t s) {
  dim3 b = lattice_block(L), g = lattice_grid(L, b);
  if (fp16) k_set_pops<__half><<<g, b, 0, s>>>(L, dst, in);
  else k_set_pops<float><<<g, b, 0, s>>>(L, dst, in);
}

// ---- tangent (forward sensitivity) of the lattice update -------------------------
// Derivative of collide + stream + walls along the tangent populations t_i,
// the tangent force density dg and the wall-speed rate duw, at the current
// FP32 populations (the product rule through the moments, the equilibrium and
// Guo's term; streaming is linear).  One node per thread.
template <bool LINEAR>
__global__ __launch_bounds__(256) void k_tangent_collide_stream(LatDev L, TanDev Tn, int src,
                                                                int par) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= L.nx || y >= L.ny) return;
  const long long S = L.S;
  const long long n0 = ((long long)z * L.ny + y) * L.nx + x;
  const float *fs = static_cast<const float *>(L.f[src]);
  const float *ts = Tn.df[src];
  float *td = Tn.df[src ^ 1];
  float d[Q], t[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    d[i] = fs[pidx(L, i, (long long)z * L.ny + y, x)];
    t[i] = ts[i * S + n0];
  }
  float gx = 0.0f, gy = 0.0f, gz = 0.0f, hx = 0.0f, hy = 0.0f, hz = 0.0f;
  const int step = L.ctrl->step;
  const int tile = tile_of(L, x, y, z);
  if (L.stamp[par][tile] == step) {
    gx = L.g[par][gix(n0, 0)];
    gy = L.g[par][gix(n0, 1)];
    gz = L.g[par][gix(n0, 2)];
    hx = Tn.dg[par][n0];
    hy = Tn.dg[par][S + n0];
    hz = Tn.dg[par][2 * S + n0];
  }
  if (L.stamp[par ^ 1][tile] == step - 1) {
    Tn.dg[par ^ 1][n0] = 0.0f;
    Tn.dg[par ^ 1][S + n0] = 0.0f;
    Tn.dg[par ^ 1][2 * S + n0] = 0.0f;
  }
  float drho = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f, trho = 0.0f, tjx = 0.0f, tjy = 0.0f, tjz = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    drho += d[i];
    trho += t[i];
    if (cx(i)) {
      jx += cx(i) * d[i];
      tjx += cx(i) * t[i];
    }
    if (cy(i)) {
      jy += cy(i) * d[i];
      tjy += cy(i) * t[i];
    }
    if (cz(i)) {
      jz += cz(i) * d[i];
      tjz += cz(i) * t[i];
    }
  }
  const float rho = 1.0f + drho, inv_rho = 1.0f / rho;
  const float ux = (jx + 0.5f * gx) * inv_rho, uy = (jy + 0.5f * gy) * inv_rho,
              uz = (jz + 0.5f * gz) * inv_rho;
  const float vx = (tjx + 0.5f * hx - ux * trho) * inv_rho;
  const float vy = (tjy + 0.5f * hy - uy * trho) * inv_rho;
  const float vz = (tjz + 0.5f * hz - uz * trho) * inv_rho;
  const float usq15 = 1.5f * (ux * ux + uy * uy + uz * uz);
  const float duu3 = 3.0f * (ux * vx + uy * vy + uz * vz);
  const float dgu = vx * gx + vy * gy + vz * gz + ux * hx + uy * hy + uz * hz;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float w = (float)wgt(i);
    const float cu = cx(i) * ux + cy(i) * uy + cz(i) * uz;
    const float dcu = cx(i) * vx + cy(i) * vy + cz(i) * vz;
    float tdeq;
    if (LINEAR) tdeq = w * (trho + trho * 3.0f * cu + rho * 3.0f * dcu);
    else
      tdeq = w * (trho + trho * (3.0f * cu + 4.5f * cu * cu - usq15) +
                  rho * (3.0f * dcu + 9.0f * cu * dcu - duu3));
    const float cg = cx(i) * gx + cy(i) * gy + cz(i) * gz;
    const float dcg = cx(i) * hx + cy(i) * hy + cz(i) * hz;
    t[i] = t[i] - (t[i] - tdeq) * L.inv_tau +
           L.guo_pre * w * (3.0f * (dcg - dgu) + 9.0f * (dcu * cg + cu * dcg));
  }
  const long long plane = (long long)L.nx * L.ny;
  const int ym = (y == 0) ? L.ny - 1 : y - 1, yp = (y == L.ny - 1) ? 0 : y + 1;
  const int xm = (x == 0) ? L.nx - 1 : x - 1, xp = (x == L.nx - 1) ? 0 : x + 1;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int zt = z + cz(i);
    if (cz(i) != 0 && (zt < 0 || zt >= L.nz)) {
      const float duwall = (zt < 0) ? -Tn.duw : Tn.duw;
      td[opp(i) * S + n0] = t[i] - 6.0f * (float)wgt(i) * (float)cx(i) * duwall;
    } else {
      const int yt = cy(i) > 0 ? yp : (cy(i) < 0 ? ym : y);
      const int xt = cx(i) > 0 ? xp : (cx(i) < 0 ? xm : x);
      td[i * S + (long long)zt * plane + (long long)yt * L.nx + xt] = t[i];
    }
  }
}

void launch_tangent_collide_stream(const LatDev &L, const TanDev &T, int src, int par, bool linear,
                                   hipStream_t s) {
  dim3 b = lattice_block(L), g = lattice_grid(L, b);
  if (linear) k_tangent_collide_stream<true><<<g, b, 0, s>>>(L, T, src, par);
  else k_tangent_collide_stream<false><<<g, b, 0, s>>>(L, T, src, par);
}

// Initial tangent populations: zero, or (profile) the derivative of the Couette
// equilibrium f_i^eq(1, u_w (2z + 1 - nz) / nz) with respect to u_w times duw.
__global__ __launch_bounds__(256) void k_tangent_init(LatDev L, TanDev Tn, int dst, int profile,
                                                      int linear) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= L.nx || y >= L.ny) return;
  const long long n = ((long long)z * L.ny + y) * L.nx + x;
  const double shape = (double)(2 * z + 1 - L.nz) / (double)L.nz;
  const double ux = (double)L.uw * shape, dux = (double)Tn.duw * shape;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    double v = 0.0;
    if (profile) {
      const double c = cx(i);
      v = linear ? wgt(i) * 3.0 * c * dux : wgt(i) * (3.0 * c + 9.0 * c * c * ux - 3.0 * ux) * dux;
    }
    Tn.df[dst][i * L.S + n] = (float)v;
  }
}

void launch_tangent_init(const LatDev &L, const TanDev &T, int dst, int profile, int linear,
                         hipStream_t s) {
  dim3 b = lattice_block(L), g = lattice_grid(L, b);
  k_tangent_init<<<g, b, 0, s>>>(L, T, dst, profile, linear);
}

// Tangent populations out, [19][nz][ny][nx] FP64.
__global__ __launch_bounds__(256) void k_get_tangent_pops(LatDev L, TanDev Tn, int src,
                                                          double *out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= L.nx || y >= L.ny) return;
  const long long N = (long long)L.nx * L.ny * L.nz;
  const long long n = ((long long)z * L.ny + y) * L.nx + x;
#pragma unroll
  for (int i = 0; i < Q; ++i) out[i * N + n] = Tn.df[src][i * L.S + n];
}

void launch_get_tangent_pops(const LatDev &L, const TanDev &T, int src, double *out,
                             hipStream_t s) {
  dim3 b = lattice_block(L), g = lattice_grid(L, b);
  k_get_tangent_pops<<<g, b, 0, s>>>(L, T, src, out);
}

// ---- adjoint (reverse mode) of the lattice part of the step -----------------------
// Reverse of one step t, given the adjoint of f(t+1) (A.lf[cur]) and of the
// lattice velocity at the stencil nodes (A.lU).  f0 and f1 are the stored
// populations f(t) and f(t+1) (same layout as the lattice buffers), g(t) is in
// L.g[par] where the tile is stamped with `step`.

// Lattice velocity U = (j(f1) + g/2) / rho(f1) at the stencil nodes: adds
// (c_i - U) . lU / rho to the adjoint of f1_i and sets the force-density
// adjoint lg = lU / (2 rho) (every node of a tile the step's stencils touch,
// A.stamp, so stale values of an older step are overwritten); clears lU.
__global__ __launch_bounds__(256) void k_adj_velocity(LatDev L, AdjDev A, const float *f1, int par,
                                                      int step, int cur) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= L.nx || y >= L.ny) return;
  if (A.stamp[tile_of(L, x, y, z)] != step) return;
  const long long S = L.S;
  const long long row = (long long)z * L.ny + y;
  const long long n = row * L.nx + x;
  const float ax = A.lU[n], ay = A.lU[S + n], az = A.lU[2 * S + n];
  if (ax == 0.0f && ay == 0.0f && az == 0.0f) {
    A.lg[n] = A.lg[S + n] = A.lg[2 * S + n] = 0.0f;
    return;
  }
  float drho = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float d = f1[pidx(L, i, row, x)];
    drho += d;
    if (cx(i)) jx += cx(i) * d;
    if (cy(i)) jy += cy(i) * d;
    if (cz(i)) jz += cz(i) * d;
  }
  const float inv_rho = 1.0f / (1.0f + drho);
  const float *g = L.g[par];
  const float ux = (jx + 0.5f * g[gix(n, 0)]) * inv_rho, uy = (jy + 0.5f * g[gix(n, 1)]) * inv_rho,
              uz = (jz + 0.5f * g[gix(n, 2)]) * inv_rho;
  const float au = ax * ux + ay * uy + az * uz;
  float *lf = A.lf[cur];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const long long at = pidx(L, i, row, x);
    lf[at] += (cx(i) * ax + cy(i) * ay + cz(i) * az - au) * inv_rho;
  }
  A.lg[n] = 0.5f * ax * inv_rho;
  A.lg[S + n] = 0.5f * ay * inv_rho;
  A.lg[2 * S + n] = 0.5f * az * inv_rho;
  A.lU[n] = A.lU[S + n] = A.lU[2 * S + n] = 0.0f;
}

void launch_adj_velocity(const LatDev &L, const AdjDev &A, const float *f1, int par, int step,
                         int cur, hipStream_t s) {
  dim3 b = lattice_block(L), g = lattice_grid(L, b);
  k_adj_velocity<<<g, b, 0, s>>>(L, A, f1, par, step, cur);
}

// Streaming (pulled back from x + c_i, or from the bounce-back partner at a
// wall), then BGK + Guo reversed at the node: with u = (j + g/2)/rho,
//   lf_k = (1 - 1/tau) l*_k + lrho + lu . (c_k - u) / rho,
//   lrho = sum_i l*_i (1/tau) d feq_i / d rho,
//   lu   = sum_i l*_i [(1/tau) d feq_i / d u + d S_i / d u],
//   lg  += sum_i l*_i d S_i / d g + lu / (2 rho)     (stencil tiles only),
// and the wall-speed term of the bounce-back kick into the per-column sums.
template <bool LINEAR>
__global__ __launch_bounds__(256) void k_adj_collide_stream(LatDev L, AdjDev A, const float *f0,
                                                            int par, int step, int cur) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= L.nx || y >= L.ny) return;
  const long long S = L.S;
  const long long row = (long long)z * L.ny + y;
  const long long n = row * L.nx + x;
  const float *l1 = A.lf[cur];
  float *l0 = A.lf[cur ^ 1];
  const int ym = (y == 0) ? L.ny - 1 : y - 1, yp = (y == L.ny - 1) ? 0 : y + 1;
  const int xm = (x == 0) ? L.nx - 1 : x - 1, xp = (x == L.nx - 1) ? 0 : x + 1;
  float ls[Q];
  float luw = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int zt = z + cz(i);
    if (cz(i) != 0 && (zt < 0 || zt >= L.nz)) {
      const float v = l1[pidx(L, opp(i), row, x)];
      ls[i] = v;
      luw += v * (-6.0f * (float)wgt(i) * (float)cx(i) * (zt < 0 ? -1.0f : 1.0f));
    } else {
      const int yt = cy(i) > 0 ? yp : (cy(i) < 0 ? ym : y);
      const int xt = cx(i) > 0 ? xp : (cx(i) < 0 ? xm : x);
      ls[i] = l1[pidx(L, i, (long long)zt * L.ny + yt, xt)];
    }
  }
  if (z == 0 || z == L.nz - 1)
    A.uw_col[(z == 0 ? 0 : (long long)L.nx * L.ny) + (long long)y * L.nx + x] += (double)luw;
  float drho = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float d = f0[pidx(L, i, row, x)];
    drho += d;
    if (cx(i)) jx += cx(i) * d;
    if (cy(i)) jy += cy(i) * d;
    if (cz(i)) jz += cz(i) * d;
  }
  // the force density is zero outside the tiles spreading touched; its
  // adjoint is needed wherever the step's stencils reach
  const bool stamped = A.stamp[tile_of(L, x, y, z)] == step;
  const float gx = L.g[par][gix(n, 0)], gy = L.g[par][gix(n, 1)], gz = L.g[par][gix(n, 2)];
  const float rho = 1.0f + drho, inv_rho = 1.0f / rho;
  const float ux = (jx + 0.5f * gx) * inv_rho, uy = (jy + 0.5f * gy) * inv_rho,
              uz = (jz + 0.5f * gz) * inv_rho;
  const float usq15 = 1.5f * (ux * ux + uy * uy + uz * uz);
  const float itau = L.inv_tau, pre = L.guo_pre;
  float lrho = 0.0f, lux = 0.0f, luy = 0.0f, luz = 0.0f, lgx = 0.0f, lgy = 0.0f, lgz = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float w = (float)wgt(i);
    const float cu = cx(i) * ux + cy(i) * uy + cz(i) * uz;
    const float Qi = LINEAR ? 3.0f * cu : 3.0f * cu + 4.5f * cu * cu - usq15;
    lrho += ls[i] * itau * w * (1.0f + Qi);
    const float a = ls[i] * itau * w * rho;
    if (LINEAR) {
      lux += a * 3.0f * cx(i);
      luy += a * 3.0f * cy(i);
      luz += a * 3.0f * cz(i);
    } else {
      lux += a * (3.0f * cx(i) + 9.0f * cu * cx(i) - 3.0f * ux);
      luy += a * (3.0f * cy(i) + 9.0f * cu * cy(i) - 3.0f * uy);
      luz += a * (3.0f * cz(i) + 9.0f * cu * cz(i) - 3.0f * uz);
    }
    if (stamped) {
      const float cg = cx(i) * gx + cy(i) * gy + cz(i) * gz;
      const float b = ls[i] * pre * w;
      lux += b * (-3.0f * gx + 9.0f * cg * cx(i));
      luy += b * (-3.0f * gy + 9.0f * cg * cy(i));
      luz += b * (-3.0f * gz + 9.0f * cg * cz(i));
      lgx += b * (3.0f * (cx(i) - ux) + 9.0f * cu * cx(i));
      lgy += b * (3.0f * (cy(i) - uy) + 9.0f * cu * cy(i));
      lgz += b * (3.0f * (cz(i) - uz) + 9.0f * cu * cz(i));
    }
  }
  const float luu = lux * ux + luy * uy + luz * uz;
#pragma unroll
  for (int k = 0; k < Q; ++k)
    l0[pidx(L, k, row, x)] =
        (1.0f - itau) * ls[k] + lrho + (lux * cx(k) + luy * cy(k) + luz * cz(k) - luu) * inv_rho;
  if (stamped) {
    A.lg[n] += lgx + 0.5f * lux * inv_rho;
    A.lg[S + n] += lgy + 0.5f * luy * inv_rho;
    A.lg[2 * S + n] += lgz + 0.5f * luz * inv_rho;
  }
}

void launch_adj_collide_stream(const LatDev &L, const AdjDev &A, const float *f0, int par, int step,
                               int cur, bool linear, hipStream_t s) {
  dim3 b = lattice_block(L), g = lattice_grid(L, b);
  if (linear) k_adj_collide_stream<true><<<g, b, 0, s>>>(L, A, f0, par, step, cur);
  else k_adj_collide_stream<false><<<g, b, 0, s>>>(L, A, f0, par, step, cur);
}

// d/du_w through the Couette start f_i(0) = f_i^eq(1, u_w (2z + 1 - nz)/nz):
// sum over the lattice of lf_i(0) d f_i(0) / d u_w, one partial sum per block.
__global__ __launch_bounds__(256) void k_adj_couette_start(LatDev L, AdjDev A, int cur, int linear,
                                                           double *partial) {
  __shared__ double red[256];
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int nt = blockDim.x * blockDim.y;
  double v = 0.0;
  if (x < L.nx && y < L.ny) {
    const long long row = (long long)z * L.ny + y;
    const double shape = (double)(2 * z + 1 - L.nz) / (double)L.nz;
    const double ux = (double)L.uw * shape;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double c = cx(i);
      const double dfi = linear ? wgt(i) * 3.0 * c * shape
                                : wgt(i) * (3.0 * c + 9.0 * c * c * ux - 3.0 * ux) * shape;
      v += (double)A.lf[cur][pidx(L, i, row, x)] * dfi;
    }
  }
  red[tid] = v;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (tid < k && tid + k < nt) red[tid] += red[tid + k];
    __syncthreads();
  }
  if (tid == 0) partial[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = red[0];
}

long long adj_couette_blocks(const LatDev &L) {
  dim3 b = lattice_block(L), g = lattice_grid(L, b);
  return (long long)g.x * g.y * g.z;
}

void launch_adj_couette_start(const LatDev &L, const AdjDev &A, int cur, int linear,
                              double *partial, hipStream_t s) {
  dim3 b = lattice_block(L), g = lattice_grid(L, b);
  k_adj_couette_start<<<g, b, 0, s>>>(L, A, cur, linear, partial);
}

// ---- batches of runs -------------------------------------------------------------
// The lattice update of many independent runs in one launch: block b updates
// part lat_items[b].y of run lat_items[b].x, four wavefronts of whole rows in
// the row form (runs whose padded rows have at most 256 values), else 256
// consecutive nodes, one per thread.  Runs without
// capsules never stamp a tile, so reading the force field only where stamped
// is correct for them as well.
template <typename T, bool LINEAR>
__global__ __launch_bounds__(256) void k_batch_collide_stream(BatchDev B, int src, int par) {
  if ((int)blockIdx.x >= B.n_lat_items) return;
  const int2 it = B.lat_items[blockIdx.x];
  // a private copy with the buffers of this step in slot 0, so that the update
  // indexes the pointer pairs with constants (registers, not scratch)
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
  if (L.tpr > 0) {
    // row form: B.wpb wavefronts of rpw whole rows per block
    const int lane = threadIdx.x & 63;
    const int wave = it.y * B.wpb + (int)(threadIdx.x >> 6);
    if (wave * L.rpw >= L.ny * L.nz) return;  // the whole wavefront is past the last row
    const int r = lane / L.tpr;
    const int t = lane - r * L.tpr;
    const int row = wave * L.rpw + r;
    // cached writes for the rows of a run below cached_rows, per wavefront
    collide_stream_rowseg<T, LINEAR, true, true>(L, 0, 0, row, t, lane, r < L.rpw && row < L.ny * L.nz,
                                                 __builtin_amdgcn_readfirstlane(row) < L.cached_rows);
    return;
  }
  // a lattice holds at most 2^31 nodes: unsigned 32-bit index arithmetic suffices
  const unsigned idx = (unsigned)it.y * blockDim.x + threadIdx.x;
  if ((long long)idx >= (long long)L.nx * L.ny * L.nz) return;
  const unsigned nx = (unsigned)L.nx, ny = (unsigned)L.ny;
  const unsigned row = idx / nx;
  collide_stream_nodes<T, LINEAR, true, 1, true>(L, 0, 0, (int)(idx - row * nx), (int)(row % ny),
                                                 (int)(row / ny));
}

void launch_batch_collide_stream(const BatchDev &B, int fp16, int src, int par, bool linear,
                                 hipStream_t s, const DispatchTimer *t) {
  if (B.n_lat_items <= 0) return;
  const dim3 grid(B.n_lat_items), block(64 * B.wpb);
  if (fp16) {
    if (linear) launch_k(k_batch_collide_stream<__half, true>, grid, block, s, t, B, src, par);
    else launch_k(k_batch_collide_stream<__half, false>, grid, block, s, t, B, src, par);
  } else {
    if (linear) launch_k(k_batch_collide_stream<float, true>, grid, block, s, t, B, src, par);
    else launch_k(k_batch_collide_stream<float, false>, grid, block, s, t, B, src, par);
  }
}

// ---- FP64 lattice totals, Eqs. (lbmmomenta0/1) summed over all nodes ---------
// Mass sum_X sum_i f_i and momentum sum_X sum_i c_i f_i of the populations in
// buffer src.  Block b sums nodes [b TOTALS_NODES, (b + 1) TOTALS_NODES) of
// the lattice order n = (z ny + y) nx + x in FP64 and writes its partial
// (sum of the deviations f_i - w_i, momentum) to part[b]; one block then adds
// the partials.  Every sum runs in a fixed order, so a state always gives the
// same bits.  The stored values are converted exactly (stored_deviation).
__device__ __forceinline__ void block_sum4(double (&v)[4]) {
  __shared__ double red[4][256];
  const int t = threadIdx.x;
#pragma unroll
  for (int c = 0; c < 4; ++c) red[c][t] = v[c];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h)
#pragma unroll
      for (int c = 0; c < 4; ++c) red[c][t] += red[c][t + h];
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) v[c] = red[c][0];
}

template <typename T>
__global__ __launch_bounds__(256) void k_totals_partial(LatDev L, int src, double4 *part) {
  const long long N = (long long)L.nx * L.ny * L.nz;
  const long long n0 = (long long)blockIdx.x * TOTALS_NODES;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < TOTALS_NODES; k += blockDim.x) {
    const long long n = n0 + k;
    if (n >= N) break;
    const long long row = n / L.nx;
    const int x = (int)(n - row * L.nx), y = (int)(row % L.ny), z = (int)(row / L.ny);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double d = stored_post<T>(L, src, i, x, y, z);
      v[0] += d;
      if (cx(i)) v[1] += cx(i) * d;
      if (cy(i)) v[2] += cy(i) * d;
      if (cz(i)) v[3] += cz(i) * d;
    }
  }
  block_sum4(v);
  if (threadIdx.x == 0) part[blockIdx.x] = make_double4(v[0], v[1], v[2], v[3]);
}

// out[0] = N + sum of the partial mass deviations (sum_i w_i = 1 per node),
// out[1..3] = momentum (sum_i c_i w_i = 0)
__global__ __launch_bounds__(256) void k_totals_final(const double4 *part, int nparts, long long N,
                                                      double *out) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < nparts; k += blockDim.x) {
    const double4 p = part[k];
    v[0] += p.x;
    v[1] += p.y;
    v[2] += p.z;
    v[3] += p.w;
  }
  block_sum4(v);
  if (threadIdx.x == 0) {
    out[0] = (double)N + v[0];
    out[1] = v[1];
    out[2] = v[2];
    out[3] = v[3];
  }
}

int totals_parts(const LatDev &L) {
  const long long N = (long long)L.nx * L.ny * L.nz;
  return (int)((N + TOTALS_NODES - 1) / TOTALS_NODES);
}

void launch_totals(const LatDev &L, int fp16, int src, double4 *part, double *out, hipStream_t s) {
  const int np = totals_parts(L);
  if (fp16) k_totals_partial<__half><<<dim3(np), dim3(256), 0, s>>>(L, src, part);
  else k_totals_partial<float><<<dim3(np), dim3(256), 0, s>>>(L, src, part);
  k_totals_final<<<dim3(1), dim3(256), 0, s>>>(part, np, (long long)L.nx * L.ny * L.nz, out);
}

// ---- fills (no hipMemset, so that the same code can be captured) --------------
__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, long long n, uint32_t v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

void launch_fill_u32(void *p, long long n, uint32_t v, hipStream_t s) {
  if (n <= 0) return;
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_fill_u32<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(static_cast<uint32_t *>(p), n, v);
}

}  // namespace ibm
