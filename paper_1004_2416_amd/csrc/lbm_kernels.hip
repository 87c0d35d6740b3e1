// Lattice kernels: fused D3Q19 BGK collision with Guo forcing, streaming and
// moving-wall bounce-back (Sec. II.A), equilibrium initialisation, and the
// FP64 field I/O of the public interface.
//
// Storage: populations as deviations d_i = f_i - w_i from the lattice weights,
// structure of arrays [19][S] (S >= nx*ny*nz, x fastest), in FP32 or in FP16
// scaled per direction.  Two buffers alternate: the kernel reads f(t) at the
// node itself (aligned loads) and pushes the post-collision values to the
// neighbours of buffer t+1, so both buffers always hold post-streaming
// populations at their own nodes.  A thread block covers whole x rows, so
// every cache line of the destination is written by one block.
#include "common.h"
#include "launch.h"

namespace ibm {

template <typename T>
__device__ __forceinline__ float ld_dev(const T *p, long long idx, float inv_scale);
template <>
__device__ __forceinline__ float ld_dev<float>(const float *p, long long idx, float) {
  return p[idx];
}
template <>
__device__ __forceinline__ float ld_dev<__half>(const __half *p, long long idx, float inv_scale) {
  return __half2float(p[idx]) * inv_scale;
}
template <typename T>
__device__ __forceinline__ void st_dev(T *p, long long idx, float v, float scale);
template <>
__device__ __forceinline__ void st_dev<float>(float *p, long long idx, float v, float) {
  p[idx] = v;
}
template <>
__device__ __forceinline__ void st_dev<__half>(__half *p, long long idx, float v, float scale) {
  p[idx] = __float2half_rn(v * scale);
}

// One lattice update at node (x, y, z) of buffer `src` into buffer src ^ 1.
//   Moments (Eqs. lbmmomenta0/1): rho = 1 + sum d_i, rho u = sum c_i d_i + g/2
//   (sum c_i w_i = 0).  Equilibrium deviation (Eq. equilibrium):
//   feq_i - w_i = w_i (rho - 1) + w_i rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u).
//   Guo term (Eq. latticeforce), BGK relaxation (Eq. lbequation), then
//   streaming to x + c_i, periodic in x and y; populations leaving through a
//   wall return to x reversed, with -2 w_i rho_w (c_i . u_wall) / c_s^2,
//   rho_w = 1 (bounce-back for moving walls).
template <typename T, bool LINEAR, bool FORCE>
__global__ __launch_bounds__(256) void k_collide_stream(LatDev L, int src, int par) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= L.nx || y >= L.ny) return;
  const long long S = L.S;
  const long long nxl = L.nx;
  const long long plane = nxl * L.ny;
  const long long n = (long long)z * plane + (long long)y * nxl + x;
  const T *__restrict__ fs = static_cast<const T *>(L.f[src]);
  T *__restrict__ fd = static_cast<T *>(L.f[src ^ 1]);

  float d[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) d[i] = ld_dev<T>(fs, i * S + n, 1.0f / L.h_scale[i]);

  float drho = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    drho += d[i];
    if (cx(i)) jx += cx(i) * d[i];
    if (cy(i)) jy += cy(i) * d[i];
    if (cz(i)) jz += cz(i) * d[i];
  }
  const float rho = 1.0f + drho;

  float gx = 0.0f, gy = 0.0f, gz = 0.0f;
  if (FORCE) {
    const int t = L.ctrl->step;
    const int tile = tile_of(L, x, y, z);
    if (L.stamp[par][tile] == t) {
      const float *g = L.g[par];
      gx = g[n];
      gy = g[S + n];
      gz = g[2 * S + n];
    }
    // The other field was spread one step ago and has been interpolated
    // from; clear it where it was touched so the next spreading starts at 0.
    if (L.stamp[par ^ 1][tile] == t - 1) {
      float *go = L.g[par ^ 1];
      go[n] = 0.0f;
      go[S + n] = 0.0f;
      go[2 * S + n] = 0.0f;
    }
  }
  const float inv_rho = 1.0f / rho;
  const float ux = (jx + 0.5f * gx) * inv_rho;
  const float uy = (jy + 0.5f * gy) * inv_rho;
  const float uz = (jz + 0.5f * gz) * inv_rho;
  const float usq15 = 1.5f * (ux * ux + uy * uy + uz * uz);
  const float gu = ux * gx + uy * gy + uz * gz;

  const int xm = (x == 0) ? L.nx - 1 : x - 1;
  const int xp = (x == L.nx - 1) ? 0 : x + 1;
  const int ym = (y == 0) ? L.ny - 1 : y - 1;
  const int yp = (y == L.ny - 1) ? 0 : y + 1;

#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float w = (float)wgt(i);
    const float cu = cx(i) * ux + cy(i) * uy + cz(i) * uz;
    float deq;
    if (LINEAR) deq = w * (drho + rho * 3.0f * cu);
    else deq = w * (drho + rho * (3.0f * cu + 4.5f * cu * cu - usq15));
    float post = d[i] - (d[i] - deq) * L.inv_tau;
    if (FORCE) {
      const float cg = cx(i) * gx + cy(i) * gy + cz(i) * gz;
      post += L.guo_pre * w * (3.0f * (cg - gu) + 9.0f * cu * cg);
    }
    const int zt = z + cz(i);
    if (cz(i) != 0 && (zt < 0 || zt >= L.nz)) {
      const float uwall = (zt < 0) ? -L.uw : L.uw;
      const float v = post - 6.0f * w * (float)cx(i) * uwall;
      st_dev<T>(fd, opp(i) * S + n, v, L.h_scale[opp(i)]);
    } else {
      const int xt = cx(i) > 0 ? xp : (cx(i) < 0 ? xm : x);
      const int yt = cy(i) > 0 ? yp : (cy(i) < 0 ? ym : y);
      const long long nt = (long long)zt * plane + (long long)yt * nxl + xt;
      st_dev<T>(fd, i * S + nt, post, L.h_scale[i]);
    }
  }
}

// Block shape: whole x rows (up to 256 nodes), stacked in y to 256 threads.
static dim3 lattice_block(const LatDev &L) {
  int bx = ((L.nx + 31) / 32) * 32;
  if (bx > 256) bx = 256;
  int by = 256 / bx;
  if (by < 1) by = 1;
  return dim3(bx, by, 1);
}

static dim3 lattice_grid(const LatDev &L, dim3 b) {
  return dim3((L.nx + b.x - 1) / b.x, (L.ny + b.y - 1) / b.y, L.nz);
}

template <typename T>
static void launch_cs_t(const LatDev &L, int src, int par, bool force, bool linear,
                        hipStream_t s) {
  dim3 b = lattice_block(L), g = lattice_grid(L, b);
  if (force) {
    if (linear) k_collide_stream<T, true, true><<<g, b, 0, s>>>(L, src, par);
    else k_collide_stream<T, false, true><<<g, b, 0, s>>>(L, src, par);
  } else {
    if (linear) k_collide_stream<T, true, false><<<g, b, 0, s>>>(L, src, par);
    else k_collide_stream<T, false, false><<<g, b, 0, s>>>(L, src, par);
  }
}

void launch_collide_stream(const LatDev &L, int fp16, int src, int par, bool force,
                           bool linear, hipStream_t s) {
  if (fp16) launch_cs_t<__half>(L, src, par, force, linear, s);
  else launch_cs_t<float>(L, src, par, force, linear, s);
}

// ---- initialisation: f = feq(rho = 1, u = (uw (2 z + 1 - nz) / nz, 0, 0)) ----
template <typename T>
__global__ __launch_bounds__(256) void k_init_equilibrium(LatDev L, int dst, double uw) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= L.nx || y >= L.ny) return;
  const long long n = ((long long)z * L.ny + y) * L.nx + x;
  const double ux = uw * (2.0 * z + 1.0 - L.nz) / L.nz;
  T *f = static_cast<T *>(L.f[dst]);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double cu = cx(i) * ux;
    const double d = wgt(i) * (3.0 * cu + 4.5 * cu * cu - 1.5 * ux * ux);
    st_dev<T>(f, i * L.S + n, (float)d, L.h_scale[i]);
  }
}

void launch_init_equilibrium(const LatDev &L, int fp16, int dst, double uw, hipStream_t s) {
  dim3 b = lattice_block(L), g = lattice_grid(L, b);
  if (fp16) k_init_equilibrium<__half><<<g, b, 0, s>>>(L, dst, uw);
  else k_init_equilibrium<float><<<g, b, 0, s>>>(L, dst, uw);
}

// ---- FP64 field I/O ----------------------------------------------------------
// what: 0 populations, 1 density, 2 velocity, 3 force density.  gpar < 0: no
// force field yet (velocity without the half-force term, force = 0).
template <typename T>
__global__ __launch_bounds__(256) void k_get_field(LatDev L, int src, int gpar, int what,
                                                   double *out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= L.nx || y >= L.ny) return;
  const long long N = (long long)L.nx * L.ny * L.nz;
  const long long n = ((long long)z * L.ny + y) * L.nx + x;
  const T *f = static_cast<const T *>(L.f[src]);
  double gx = 0.0, gy = 0.0, gz = 0.0;
  if (gpar >= 0) {
    const float *g = L.g[gpar];
    gx = g[n];
    gy = g[L.S + n];
    gz = g[2 * L.S + n];
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
    const double d = ld_dev<T>(f, i * L.S + n, 1.0f / L.h_scale[i]);
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
  for (int i = 0; i < Q; ++i) st_dev<T>(f, i * L.S + n, (float)(in[i * N + n] - wgt(i)), L.h_scale[i]);
}

void launch_set_pops(const LatDev &L, int fp16, int dst, const double *in, hipStream_t s) {
  dim3 b = lattice_block(L), g = lattice_grid(L, b);
  if (fp16) k_set_pops<__half><<<g, b, 0, s>>>(L, dst, in);
  else k_set_pops<float><<<g, b, 0, s>>>(L, dst, in);
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
