// Host runtime behind the C ABI declared in include/ibm_lbm.h: handle state,
// carving of the caller's device buffers, validation, the per-step kernel
// sequence (Sec. II.C sub-steps 1-5), hipGraph replay, profiling and errors.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ibm_lbm.h"
#include "common.h"
#include "launch.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int ok() {
  g_last_error.clear();
  return IBM_OK;
}

#define IBM_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(IBM_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));         \
  } while (0)

constexpr size_t ALIGN = 256;
size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Steps replayed per graph launch (even, so that the buffer parity returns).
constexpr int GRAPH_STEPS = 16;

struct LatticeLayout {
  long long N, S;
  int tnx, tny, tnz;
  size_t off_ctrl, off_stamp[2], off_g[2], off_f[2], total;
};

LatticeLayout lattice_layout(int nx, int ny, int nz, int storage) {
  LatticeLayout l{};
  l.N = (long long)nx * ny * nz;
  l.S = (long long)round_up((size_t)l.N, 64);
  l.tnx = (nx + ibm::TILE_X - 1) / ibm::TILE_X;
  l.tny = (ny + ibm::TILE_Y - 1) / ibm::TILE_Y;
  l.tnz = (nz + ibm::TILE_Z - 1) / ibm::TILE_Z;
  const size_t tiles = (size_t)l.tnx * l.tny * l.tnz;
  const size_t es = storage == IBM_STORAGE_FP16 ? 2 : 4;
  size_t off = 0;
  l.off_ctrl = off;
  off += round_up(sizeof(ibm::Ctrl), ALIGN);
  for (int k = 0; k < 2; ++k) {
    l.off_stamp[k] = off;
    off += round_up(tiles * sizeof(int), ALIGN);
  }
  for (int k = 0; k < 2; ++k) {
    l.off_g[k] = off;
    off += round_up(3 * (size_t)l.S * sizeof(float), ALIGN);
  }
  for (int k = 0; k < 2; ++k) {
    l.off_f[k] = off;
    off += round_up((size_t)ibm::Q * l.S * es, ALIGN);
  }
  l.total = off;
  return l;
}

struct MembraneLayout {
  size_t x, u, F, face_grad, ext_id, node_cap, csr_off, csr_ent, tri, ref_p, ref_ghi, ref_glo, origin, moduli,
      cap_node_off, cap_face_off, obs, total;
};

MembraneLayout membrane_layout(int nc, long long nn, long long nf) {
  MembraneLayout l{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += round_up(bytes, ALIGN);
    return at;
  };
  l.x = take(nn * 16);
  l.u = take(nn * 16);
  l.F = take(nn * 16);
  l.face_grad = take(3 * nf * 16);
  l.ext_id = take(nn * 4);
  l.node_cap = take(nn * 4);
  l.csr_off = take((nn + 1) * 4);
  l.csr_ent = take(3 * nf * 4);
  l.tri = take(nf * 16);
  l.ref_p = take(nf * 16);
  l.ref_ghi = take(nf * 16);
  l.ref_glo = take(nf * 16);
  l.origin = take((size_t)nc * 16);
  l.moduli = take((size_t)nc * 16);
  l.cap_node_off = take(((size_t)nc + 1) * 4);
  l.cap_face_off = take(((size_t)nc + 1) * 4);
  l.obs = take((size_t)nc * IBM_OBS_N * 8);
  l.total = off;
  return l;
}

}  // namespace

struct ibm_lattice {
  int nx = 0, ny = 0, nz = 0, storage = 0;
  double tau = 1.0, uw = 0.0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
  char *base = nullptr;
  LatticeLayout lay{};
  ibm::LatDev L{};
  int64_t steps = 0;  // completed timesteps; buffer steps & 1 holds f(t)

  bool has_mem = false;
  ibm::MemDev M{};
  std::vector<int> node_off, face_off;
  std::vector<int> int_of_ext;  // caller's node index -> internal (sorted) index

  // default collide-stream form: whole-row vectors where the row fits a
  // wavefront, else two nodes per thread, non-temporal, 128-thread blocks
  int use_graph = 1, eq_linear = 0, ab2 = 0, recenter_every = 64, lbm_variant = 16 | 7;
  bool have_prev_u = false;
  int64_t since_recenter = 0;

  hipGraphExec_t gexec = nullptr;
  bool graph_valid = false;
};

namespace {

void invalidate_graph(ibm_lattice *lat) {
  if (lat->gexec) (void)hipGraphExecDestroy(lat->gexec);
  lat->gexec = nullptr;
  lat->graph_valid = false;
}

// Clear the control words, the tile stamps and both force fields.
void reset_force_state(ibm_lattice *lat, hipStream_t s) {
  ibm::launch_fill_u32(lat->base + lat->lay.off_ctrl, sizeof(ibm::Ctrl) / 4, 0u, s);
  const long long tiles = (long long)lat->lay.tnx * lat->lay.tny * lat->lay.tnz;
  for (int k = 0; k < 2; ++k) {
    ibm::launch_fill_u32(lat->L.stamp[k], tiles, (uint32_t)(-100), s);
    ibm::launch_fill_u32(lat->L.g[k], 3 * lat->lay.S, 0u, s);
  }
}

// Enqueue one full timestep on stream s (Sec. II.C, sub-steps 1-5).
void enqueue_step(ibm_lattice *lat, hipStream_t s, int advect) {
  const int src = (int)(lat->steps & 1);
  const int par = src;  // force field of this step's parity
  if (lat->has_mem) {
    ibm::launch_face_gradients(lat->M, lat->L.ctrl, s);                  // 1: F(t)
    ibm::launch_spread(lat->L, lat->M, par, s);                          // 2: f(X, t)
    ibm::launch_collide_stream(lat->L, lat->storage, src, par, true,     // 3: f_i(t+1)
                               lat->eq_linear != 0, lat->lbm_variant, s);
    ibm::launch_interp_advect(lat->L, lat->M, lat->storage, src ^ 1,     // 4, 5
                              par, advect, s);
  } else {
    ibm::launch_collide_stream(lat->L, lat->storage, src, par, false, lat->eq_linear != 0,
                               lat->lbm_variant, s);
  }
  lat->steps += 1;
  lat->since_recenter += 1;
}

int advect_mode(ibm_lattice *lat) { return (lat->ab2 && lat->have_prev_u) ? 1 : 0; }

int capture_graph(ibm_lattice *lat) {
  invalidate_graph(lat);
  if (!lat->cap_stream) IBM_HIP(hipStreamCreateWithFlags(&lat->cap_stream, hipStreamNonBlocking));
  const int64_t saved_steps = lat->steps, saved_since = lat->since_recenter;
  hipGraph_t graph = nullptr;
  IBM_HIP(hipStreamBeginCapture(lat->cap_stream, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < GRAPH_STEPS; ++k) enqueue_step(lat, lat->cap_stream, advect_mode(lat));
  hipError_t e = hipStreamEndCapture(lat->cap_stream, &graph);
  lat->steps = saved_steps;
  lat->since_recenter = saved_since;
  if (e != hipSuccess) return fail(IBM_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&lat->gexec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    lat->gexec = nullptr;
    return fail(IBM_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
  }
  lat->graph_valid = true;
  return IBM_OK;
}

// Read and clear the device error flags (waits for the stream).
int check_device(ibm_lattice *lat) {
  IBM_HIP(hipStreamSynchronize(lat->stream));
  int err = 0;
  IBM_HIP(hipMemcpy(&err, &lat->L.ctrl->err, sizeof(int), hipMemcpyDeviceToHost));
  if (err) {
    int zero = 0;
    IBM_HIP(hipMemcpy(&lat->L.ctrl->err, &zero, sizeof(int), hipMemcpyHostToDevice));
    if (err & ibm::ERR_WALL)
      return fail(IBM_ERR_STENCIL_HITS_WALL, "a delta stencil reached beyond a wall");
    if (err & ibm::ERR_FACE)
      return fail(IBM_ERR_INVERTED_FACE, "a membrane face degenerated (det C <= 0)");
    if (err & ibm::ERR_NONFINITE) return fail(IBM_ERR_NONFINITE, "non-finite observables");
  }
  return IBM_OK;
}

bool finite_all(const double *v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// Integer origin floor(mean) of each capsule and FP32 coordinates relative to
// it, stored at the nodes' internal positions; checks that every stencil
// weight stays between the walls.  xyz is in the caller's node order.
int frame_positions(const ibm_lattice *lat, const double *xyz, std::vector<float4> &xl,
                    std::vector<int4> &org) {
  const int nc = (int)lat->node_off.size() - 1;
  const int nn = lat->node_off.back();
  xl.resize(nn);
  org.resize(nc);
  const double half = 0.5 * lat->M.m;
  for (int c = 0; c < nc; ++c) {
    const int n0 = lat->node_off[c], n1 = lat->node_off[c + 1];
    double s[3] = {0.0, 0.0, 0.0};
    for (int n = n0; n < n1; ++n)
      for (int d = 0; d < 3; ++d) s[d] += xyz[3 * (size_t)n + d];
    int o[3];
    for (int d = 0; d < 3; ++d) o[d] = (int)std::floor(s[d] / (n1 - n0));
    org[c] = make_int4(o[0], o[1], o[2], 0);
    for (int n = n0; n < n1; ++n) {
      float v[3];
      for (int d = 0; d < 3; ++d) v[d] = (float)(xyz[3 * (size_t)n + d] - o[d]);
      xl[lat->int_of_ext[n]] = make_float4(v[0], v[1], v[2], 0.0f);
      // lattice nodes Z with |Z - z| < m/2 carry weight: all must lie in [0, nz)
      const double z = (double)o[2] + (double)v[2];
      if (!(z > half - 1.0) || !(z < lat->nz - half))
        return fail(IBM_ERR_STENCIL_HITS_WALL,
                    "capsule %d node %d at z = %.6g: the %d-point stencil reaches a wall", c,
                    n - n0, z, lat->M.m);
    }
  }
  return IBM_OK;
}

// Order of a capsule's nodes along a Morton (Z-order) curve through their
// bounding box, so that consecutive nodes are spatial neighbours.
std::vector<int> morton_order(const double *xyz, int n) {
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int k = 0; k < n; ++k)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], xyz[3 * (size_t)k + d]);
      hi[d] = std::max(hi[d], xyz[3 * (size_t)k + d]);
    }
  std::vector<std::pair<uint32_t, int>> key(n);
  for (int k = 0; k < n; ++k) {
    uint32_t code = 0;
    uint32_t q[3];
    for (int d = 0; d < 3; ++d) {
      const double span = hi[d] - lo[d] > 0 ? hi[d] - lo[d] : 1.0;
      q[d] = (uint32_t)std::min(1023.0, std::floor((xyz[3 * (size_t)k + d] - lo[d]) / span * 1024.0));
    }
    for (int b = 9; b >= 0; --b)
      for (int d = 0; d < 3; ++d) code = (code << 1) | ((q[d] >> b) & 1u);
    key[k] = {code, k};
  }
  std::sort(key.begin(), key.end());
  std::vector<int> order(n);
  for (int k = 0; k < n; ++k) order[k] = key[k].second;
  return order;
}

}  // namespace

extern "C" {

const char *ibm_last_error(void) { return g_last_error.c_str(); }

int ibm_lattice_bytes(int nx, int ny, int nz, int storage, size_t *bytes) {
  if (!bytes) return fail(IBM_ERR_INVALID_ARG, "bytes is NULL");
  if (nx < 1 || ny < 1 || nz < 1) return fail(IBM_ERR_INVALID_ARG, "lattice size must be >= 1");
  if ((long long)nx * ny * nz > (1LL << 31))
    return fail(IBM_ERR_INVALID_ARG, "lattice larger than 2^31 nodes");
  if (nz > 65535 || ny > 65535 * 8) return fail(IBM_ERR_INVALID_ARG, "ny or nz beyond the launch grid");
  if (storage != IBM_STORAGE_FP32 && storage != IBM_STORAGE_FP16)
    return fail(IBM_ERR_INVALID_ARG, "unknown storage %d", storage);
  *bytes = lattice_layout(nx, ny, nz, storage).total;
  return ok();
}

int ibm_lattice_create(int nx, int ny, int nz, double tau, int storage, void *dev_state,
                       size_t bytes, void *stream, ibm_lattice **out) {
  if (!out) return fail(IBM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  int rc = ibm_lattice_bytes(nx, ny, nz, storage, &need);
  if (rc) return rc;
  if (!(tau > 0.5) || !std::isfinite(tau)) return fail(IBM_ERR_INVALID_ARG, "tau must be > 1/2");
  if (!dev_state) return fail(IBM_ERR_INVALID_ARG, "dev_state is NULL");
  if (((uintptr_t)dev_state) % ALIGN) return fail(IBM_ERR_INVALID_ARG, "dev_state not 256-byte aligned");
  if (bytes < need) return fail(IBM_ERR_INVALID_ARG, "dev_state has %zu bytes, %zu needed", bytes, need);

  ibm_lattice *lat = new ibm_lattice();
  lat->nx = nx;
  lat->ny = ny;
  lat->nz = nz;
  lat->storage = storage;
  lat->tau = tau;
  lat->stream = static_cast<hipStream_t>(stream);
  lat->base = static_cast<char *>(dev_state);
  lat->lay = lattice_layout(nx, ny, nz, storage);
  ibm::LatDev &L = lat->L;
  L.nx = nx;
  L.ny = ny;
  L.nz = nz;
  L.tnx = lat->lay.tnx;
  L.tny = lat->lay.tny;
  L.tnz = lat->lay.tnz;
  L.S = lat->lay.S;
  for (int k = 0; k < 2; ++k) {
    L.f[k] = lat->base + lat->lay.off_f[k];
    L.g[k] = reinterpret_cast<float *>(lat->base + lat->lay.off_g[k]);
    L.stamp[k] = reinterpret_cast<int *>(lat->base + lat->lay.off_stamp[k]);
  }
  L.ctrl = reinterpret_cast<ibm::Ctrl *>(lat->base + lat->lay.off_ctrl);
  L.inv_tau = (float)(1.0 / tau);
  L.guo_pre = (float)(1.0 - 0.5 / tau);
  L.uw = 0.0f;
  for (int i = 0; i < ibm::Q; ++i) L.h_scale[i] = 1.0f;
  if (storage == IBM_STORAGE_FP16) {
    // Deviations f_i - w_i scaled by 2^k / w_i keep a shear-flow population
    // (|f_i - w_i| <~ 0.1 w_i) in FP16's normal range with 11 significant bits.
    for (int i = 0; i < ibm::Q; ++i) L.h_scale[i] = (float)(16.0 / ibm::wgt(i));
  }
  reset_force_state(lat, lat->stream);
  for (int k = 0; k < 2; ++k) {
    const size_t words = ((size_t)ibm::Q * lat->lay.S * (storage == IBM_STORAGE_FP16 ? 2 : 4)) / 4;
    ibm::launch_fill_u32(L.f[k], (long long)words, 0u, lat->stream);  // at rest: f_i = w_i
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(lat->stream);
  if (e != hipSuccess) {
    delete lat;
    return fail(IBM_ERR_HIP, "lattice initialisation failed: %s", hipGetErrorString(e));
  }
  *out = lat;
  return ok();
}

int ibm_set_shear(ibm_lattice *lat, double u_w, int init_profile) {
  if (!lat) return fail(IBM_ERR_INVALID_ARG, "lat is NULL");
  if (!std::isfinite(u_w) || std::fabs(u_w) >= 0.3)
    return fail(IBM_ERR_INVALID_ARG, "|u_w| must be < 0.3 (low Mach number)");
  lat->uw = u_w;
  lat->L.uw = (float)u_w;
  invalidate_graph(lat);
  if (init_profile) {
    lat->steps = 0;
    lat->since_recenter = 0;
    lat->have_prev_u = false;
    reset_force_state(lat, lat->stream);
    ibm::launch_init_equilibrium(lat->L, lat->storage, 0, u_w, lat->stream);
    IBM_HIP(hipGetLastError());
  }
  return ok();
}

int ibm_membrane_bytes(int n_caps, const int *nodes_per_cap, const int *faces_per_cap,
                       size_t *bytes) {
  if (!bytes || !nodes_per_cap || !faces_per_cap) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  if (n_caps < 1) return fail(IBM_ERR_INVALID_ARG, "n_caps must be >= 1");
  long long nn = 0, nf = 0;
  for (int c = 0; c < n_caps; ++c) {
    if (nodes_per_cap[c] < 3 || faces_per_cap[c] < 1)
      return fail(IBM_ERR_INVALID_ARG, "capsule %d: too few nodes or faces", c);
    nn += nodes_per_cap[c];
    nf += faces_per_cap[c];
  }
  if (nn > (1LL << 24) || nf > (1LL << 26)) return fail(IBM_ERR_INVALID_ARG, "membrane too large");
  *bytes = membrane_layout(n_caps, nn, nf).total;
  return ok();
}

int ibm_membrane_create(ibm_lattice *lat, int n_caps, const int *nodes_per_cap,
                        const int *faces_per_cap, const double *xyz, const int32_t *tri,
                        const double *ks, const double *ka, int m, void *dev_mem, size_t bytes) {
  if (!lat) return fail(IBM_ERR_INVALID_ARG, "lat is NULL");
  if (lat->has_mem) return fail(IBM_ERR_BAD_STATE, "a membrane is already attached");
  size_t need = 0;
  int rc = ibm_membrane_bytes(n_caps, nodes_per_cap, faces_per_cap, &need);
  if (rc) return rc;
  if (!xyz || !tri || !ks || !ka || !dev_mem) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  if (m < 2 || m > 4) return fail(IBM_ERR_INVALID_ARG, "delta width m must be 2, 3 or 4");
  if (lat->nx < m || lat->ny < m)
    return fail(IBM_ERR_INVALID_ARG, "nx and ny must be at least the delta width %d", m);
  if (((uintptr_t)dev_mem) % ALIGN) return fail(IBM_ERR_INVALID_ARG, "dev_mem not 256-byte aligned");
  if (bytes < need) return fail(IBM_ERR_INVALID_ARG, "dev_mem has %zu bytes, %zu needed", bytes, need);

  std::vector<int> node_off(n_caps + 1, 0), face_off(n_caps + 1, 0);
  for (int c = 0; c < n_caps; ++c) {
    node_off[c + 1] = node_off[c] + nodes_per_cap[c];
    face_off[c + 1] = face_off[c] + faces_per_cap[c];
    if (!std::isfinite(ks[c]) || !std::isfinite(ka[c]) || ks[c] < 0 || ka[c] < 0)
      return fail(IBM_ERR_INVALID_ARG, "capsule %d: moduli must be finite and >= 0", c);
  }
  const int nn = node_off[n_caps], nf = face_off[n_caps];
  if (!finite_all(xyz, 3 * (size_t)nn)) return fail(IBM_ERR_INVALID_ARG, "non-finite node position");

  // internal node order: each capsule's nodes sorted along a Morton curve
  std::vector<int> ext_of_int(nn), int_of_ext(nn);
  for (int c = 0; c < n_caps; ++c) {
    const int n0 = node_off[c];
    const std::vector<int> order = morton_order(xyz + 3 * (size_t)n0, nodes_per_cap[c]);
    for (int k = 0; k < nodes_per_cap[c]; ++k) {
      ext_of_int[n0 + k] = n0 + order[k];
      int_of_ext[n0 + order[k]] = n0 + k;
    }
  }
  // faces with global internal node ids and the node -> (face, corner) lists
  std::vector<int4> t4(nf);
  std::vector<int> deg(nn, 0), node_cap(nn);
  std::vector<int> cap_node_off(node_off), cap_face_off(face_off);
  for (int c = 0; c < n_caps; ++c) {
    for (int n = node_off[c]; n < node_off[c + 1]; ++n) node_cap[n] = c;
    for (int j = face_off[c]; j < face_off[c + 1]; ++j) {
      int g[3];
      for (int k = 0; k < 3; ++k) {
        const int v = tri[3 * (size_t)j + k];
        if (v < 0 || v >= nodes_per_cap[c])
          return fail(IBM_ERR_INVALID_ARG, "capsule %d face %d: node index %d out of range", c,
                      j - face_off[c], v);
        g[k] = int_of_ext[node_off[c] + v];
      }
      if (g[0] == g[1] || g[1] == g[2] || g[0] == g[2])
        return fail(IBM_ERR_INVALID_ARG, "capsule %d face %d repeats a node", c, j - face_off[c]);
      t4[j] = make_int4(g[0], g[1], g[2], c);
      for (int k = 0; k < 3; ++k) deg[g[k]]++;
    }
  }
  std::vector<int> csr_off(nn + 1, 0), csr_ent(3 * (size_t)nf), fillp(nn);
  for (int n = 0; n < nn; ++n) csr_off[n + 1] = csr_off[n] + deg[n];
  for (int n = 0; n < nn; ++n) fillp[n] = csr_off[n];
  for (int j = 0; j < nf; ++j) {
    const int g[3] = {t4[j].x, t4[j].y, t4[j].z};
    for (int k = 0; k < 3; ++k) csr_ent[fillp[g[k]]++] = j * 4 + k;
  }
  std::vector<float4> mod(n_caps);
  for (int c = 0; c < n_caps; ++c) mod[c] = make_float4((float)ks[c], (float)ka[c], 0.0f, 0.0f);

  // device views
  const MembraneLayout ml = membrane_layout(n_caps, nn, nf);
  char *b = static_cast<char *>(dev_mem);
  ibm::MemDev &M = lat->M;
  M.n_caps = n_caps;
  M.nn = nn;
  M.nf = nf;
  M.m = m;
  M.x = reinterpret_cast<float4 *>(b + ml.x);
  M.u = reinterpret_cast<float4 *>(b + ml.u);
  M.F = reinterpret_cast<float4 *>(b + ml.F);
  M.face_grad = reinterpret_cast<float4 *>(b + ml.face_grad);
  M.ext_id = reinterpret_cast<int *>(b + ml.ext_id);

  M.node_cap = reinterpret_cast<int *>(b + ml.node_cap);
  M.csr_off = reinterpret_cast<int *>(b + ml.csr_off);
  M.csr_ent = reinterpret_cast<int *>(b + ml.csr_ent);
  M.tri = reinterpret_cast<int4 *>(b + ml.tri);
  M.ref_p = reinterpret_cast<float4 *>(b + ml.ref_p);
  M.ref_ghi = reinterpret_cast<float4 *>(b + ml.ref_ghi);
  M.ref_glo = reinterpret_cast<float4 *>(b + ml.ref_glo);
  M.origin = reinterpret_cast<int4 *>(b + ml.origin);
  M.moduli = reinterpret_cast<float4 *>(b + ml.moduli);
  M.cap_node_off = reinterpret_cast<int *>(b + ml.cap_node_off);
  M.cap_face_off = reinterpret_cast<int *>(b + ml.cap_face_off);
  M.obs = reinterpret_cast<double *>(b + ml.obs);
  lat->node_off = node_off;
  lat->face_off = face_off;
  lat->int_of_ext = int_of_ext;

  std::vector<float4> xl;
  std::vector<int4> org;
  rc = frame_positions(lat, xyz, xl, org);
  if (rc) {
    lat->M = ibm::MemDev{};
    lat->node_off.clear();
    lat->face_off.clear();
    return rc;
  }
  hipStream_t s = lat->stream;
  IBM_HIP(hipMemcpyAsync(M.x, xl.data(), nn * sizeof(float4), hipMemcpyHostToDevice, s));
  IBM_HIP(hipMemcpyAsync(M.node_cap, node_cap.data(), nn * sizeof(int), hipMemcpyHostToDevice, s));
  IBM_HIP(hipMemcpyAsync(M.ext_id, ext_of_int.data(), nn * sizeof(int), hipMemcpyHostToDevice, s));
  IBM_HIP(hipMemcpyAsync(M.csr_off, csr_off.data(), (nn + 1) * sizeof(int), hipMemcpyHostToDevice, s));
  IBM_HIP(hipMemcpyAsync(M.csr_ent, csr_ent.data(), 3 * (size_t)nf * sizeof(int), hipMemcpyHostToDevice, s));
  IBM_HIP(hipMemcpyAsync(M.tri, t4.data(), nf * sizeof(int4), hipMemcpyHostToDevice, s));
  IBM_HIP(hipMemcpyAsync(M.origin, org.data(), n_caps * sizeof(int4), hipMemcpyHostToDevice, s));
  IBM_HIP(hipMemcpyAsync(M.moduli, mod.data(), n_caps * sizeof(float4), hipMemcpyHostToDevice, s));
  IBM_HIP(hipMemcpyAsync(M.cap_node_off, cap_node_off.data(), (n_caps + 1) * sizeof(int), hipMemcpyHostToDevice, s));
  IBM_HIP(hipMemcpyAsync(M.cap_face_off, cap_face_off.data(), (n_caps + 1) * sizeof(int), hipMemcpyHostToDevice, s));
  ibm::launch_fill_u32(M.u, 4LL * nn, 0u, s);
  ibm::launch_fill_u32(M.F, 4LL * nn, 0u, s);
  ibm::launch_fill_u32(M.face_grad, 12LL * nf, 0u, s);
  ibm::launch_reference_geometry(M, lat->L.ctrl, s);
  IBM_HIP(hipGetLastError());
  IBM_HIP(hipStreamSynchronize(s));  // host vectors must outlive the copies
  lat->has_mem = true;
  rc = check_device(lat);
  if (rc) {
    lat->has_mem = false;
    return rc;
  }
  // the force bookkeeping restarts with the membrane
  reset_force_state(lat, s);
  lat->have_prev_u = false;
  lat->since_recenter = 0;
  invalidate_graph(lat);
  IBM_HIP(hipStreamSynchronize(s));
  return ok();
}

int ibm_step(ibm_lattice *lat, int64_t n) {
  if (!lat) return fail(IBM_ERR_INVALID_ARG, "lat is NULL");
  if (n < 0) return fail(IBM_ERR_INVALID_ARG, "negative step count");
  while (n > 0) {
    if (lat->has_mem && lat->since_recenter >= lat->recenter_every) {
      ibm::launch_recenter(lat->M, lat->stream);
      lat->since_recenter = 0;
    }
    const bool graph_ok = lat->use_graph && (lat->steps & 1) == 0 && n >= GRAPH_STEPS &&
                          (!lat->has_mem || lat->since_recenter + GRAPH_STEPS <= lat->recenter_every) &&
                          (!lat->ab2 || lat->have_prev_u);
    if (graph_ok) {
      if (!lat->graph_valid) {
        int rc = capture_graph(lat);
        if (rc) return rc;
      }
      IBM_HIP(hipGraphLaunch(lat->gexec, lat->stream));
      lat->steps += GRAPH_STEPS;
      lat->since_recenter += GRAPH_STEPS;
      n -= GRAPH_STEPS;
    } else {
      const int mode = advect_mode(lat);
      enqueue_step(lat, lat->stream, mode);
      if (lat->ab2 && lat->has_mem) lat->have_prev_u = true;
      n -= 1;
    }
  }
  IBM_HIP(hipGetLastError());
  return ok();
}

int64_t ibm_step_count(const ibm_lattice *lat) { return lat ? lat->steps : -1; }

int ibm_get_fields(ibm_lattice *lat, int what, double *dst_dev) {
  if (!lat || !dst_dev) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  if (what < IBM_FIELD_POPS || what > IBM_FIELD_FORCE) return fail(IBM_ERR_INVALID_ARG, "unknown field %d", what);
  const int src = (int)(lat->steps & 1);
  const int gpar = (lat->has_mem && lat->steps > 0) ? (int)((lat->steps - 1) & 1) : -1;
  ibm::launch_get_field(lat->L, lat->storage, src, gpar, what, dst_dev, lat->stream);
  IBM_HIP(hipGetLastError());
  int rc = check_device(lat);
  return rc ? rc : ok();
}

int ibm_set_fields(ibm_lattice *lat, int what, const double *src_dev) {
  if (!lat || !src_dev) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  if (what != IBM_FIELD_POPS) return fail(IBM_ERR_INVALID_ARG, "only the populations can be set");
  ibm::launch_set_pops(lat->L, lat->storage, (int)(lat->steps & 1), src_dev, lat->stream);
  IBM_HIP(hipGetLastError());
  return ok();
}

int ibm_get_mesh(ibm_lattice *lat, double *xyz_dev, double *force_dev, double *vel_dev) {
  if (!lat) return fail(IBM_ERR_INVALID_ARG, "lat is NULL");
  if (!lat->has_mem) return fail(IBM_ERR_BAD_STATE, "no membrane attached");
  ibm::launch_get_mesh(lat->M, xyz_dev, force_dev, vel_dev, lat->stream);
  IBM_HIP(hipGetLastError());
  int rc = check_device(lat);
  return rc ? rc : ok();
}

int ibm_set_mesh(ibm_lattice *lat, const double *xyz_host) {
  if (!lat || !xyz_host) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  if (!lat->has_mem) return fail(IBM_ERR_BAD_STATE, "no membrane attached");
  const int nn = lat->M.nn;
  if (!finite_all(xyz_host, 3 * (size_t)nn)) return fail(IBM_ERR_INVALID_ARG, "non-finite node position");
  std::vector<float4> xl;
  std::vector<int4> org;
  int rc = frame_positions(lat, xyz_host, xl, org);
  if (rc) return rc;
  IBM_HIP(hipMemcpyAsync(lat->M.x, xl.data(), nn * sizeof(float4), hipMemcpyHostToDevice, lat->stream));
  IBM_HIP(hipMemcpyAsync(lat->M.origin, org.data(), lat->M.n_caps * sizeof(int4), hipMemcpyHostToDevice, lat->stream));
  IBM_HIP(hipStreamSynchronize(lat->stream));
  lat->have_prev_u = false;
  lat->since_recenter = 0;
  return ok();
}

int ibm_observables(ibm_lattice *lat, double *out_host) {
  if (!lat || !out_host) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  if (!lat->has_mem) return fail(IBM_ERR_BAD_STATE, "no membrane attached");
  ibm::launch_observables(lat->M, lat->L.ctrl, lat->stream);
  IBM_HIP(hipGetLastError());
  IBM_HIP(hipMemcpyAsync(out_host, lat->M.obs, (size_t)lat->M.n_caps * IBM_OBS_N * sizeof(double),
                         hipMemcpyDeviceToHost, lat->stream));
  int rc = check_device(lat);
  return rc ? rc : ok();
}

int ibm_synchronize(ibm_lattice *lat) {
  if (!lat) return fail(IBM_ERR_INVALID_ARG, "lat is NULL");
  int rc = check_device(lat);
  return rc ? rc : ok();
}

int ibm_set_option(ibm_lattice *lat, int option, int value) {
  if (!lat) return fail(IBM_ERR_INVALID_ARG, "lat is NULL");
  switch (option) {
    case IBM_OPT_GRAPH:
      if (value != 0 && value != 1) return fail(IBM_ERR_INVALID_ARG, "graph option is 0 or 1");
      lat->use_graph = value;
      break;
    case IBM_OPT_EQUILIBRIUM:
      if (value != IBM_EQ_QUADRATIC && value != IBM_EQ_LINEAR)
        return fail(IBM_ERR_INVALID_ARG, "unknown equilibrium %d", value);
      lat->eq_linear = value;
      break;
    case IBM_OPT_ADVECTION:
      if (value != 0 && value != 1) return fail(IBM_ERR_INVALID_ARG, "advection is 0 or 1");
      lat->ab2 = value;
      lat->have_prev_u = false;
      break;
    case IBM_OPT_RECENTER:
      if (value < 1) return fail(IBM_ERR_INVALID_ARG, "recentre interval must be >= 1");
      lat->recenter_every = value;
      break;
    case IBM_OPT_LBM_VARIANT:
      if (value < 0 || value > 31) return fail(IBM_ERR_INVALID_ARG, "variant is 0..31");
      lat->lbm_variant = value;
      break;
    default:
      return fail(IBM_ERR_INVALID_ARG, "unknown option %d", option);
  }
  invalidate_graph(lat);
  return ok();
}

int ibm_profile_step(ibm_lattice *lat, int64_t n, double *ms_per_phase) {
  if (!lat || !ms_per_phase) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  if (n < 1 || n > 4096) return fail(IBM_ERR_INVALID_ARG, "profile 1..4096 steps");
  const int ne = lat->has_mem ? 5 : 2;
  std::vector<hipEvent_t> ev((size_t)n * ne);
  for (auto &e : ev) IBM_HIP(hipEventCreate(&e));
  hipStream_t s = lat->stream;
  for (int64_t k = 0; k < n; ++k) {
    hipEvent_t *e = &ev[(size_t)k * ne];
    const int src = (int)(lat->steps & 1), par = src;
    IBM_HIP(hipEventRecord(e[0], s));
    if (lat->has_mem) {
      ibm::launch_face_gradients(lat->M, lat->L.ctrl, s);
      IBM_HIP(hipEventRecord(e[1], s));
      ibm::launch_spread(lat->L, lat->M, par, s);
      IBM_HIP(hipEventRecord(e[2], s));
      ibm::launch_collide_stream(lat->L, lat->storage, src, par, true, lat->eq_linear != 0,
                                 lat->lbm_variant, s);
      IBM_HIP(hipEventRecord(e[3], s));
      ibm::launch_interp_advect(lat->L, lat->M, lat->storage, src ^ 1, par, advect_mode(lat), s);
      IBM_HIP(hipEventRecord(e[4], s));
      if (lat->ab2) lat->have_prev_u = true;
    } else {
      ibm::launch_collide_stream(lat->L, lat->storage, src, par, false, lat->eq_linear != 0,
                                 lat->lbm_variant, s);
      IBM_HIP(hipEventRecord(e[1], s));
    }
    lat->steps += 1;
    lat->since_recenter += 1;
  }
  IBM_HIP(hipGetLastError());
  IBM_HIP(hipStreamSynchronize(s));
  double acc[IBM_N_PHASES] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t k = 0; k < n; ++k) {
    hipEvent_t *e = &ev[(size_t)k * ne];
    float ms = 0.0f;
    if (lat->has_mem) {
      for (int p = 0; p < 4; ++p) {
        IBM_HIP(hipEventElapsedTime(&ms, e[p], e[p + 1]));
        acc[p] += ms;
      }
    } else {
      IBM_HIP(hipEventElapsedTime(&ms, e[0], e[1]));
      acc[IBM_PHASE_LBM] += ms;
    }
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  for (int p = 0; p < IBM_N_PHASES; ++p) ms_per_phase[p] = acc[p] / (double)n;
  int rc = check_device(lat);
  return rc ? rc : ok();
}

int ibm_destroy(ibm_lattice *lat) {
  if (!lat) return ok();
  (void)hipStreamSynchronize(lat->stream);
  invalidate_graph(lat);
  if (lat->cap_stream) (void)hipStreamDestroy(lat->cap_stream);
  delete lat;
  return ok();
}

}  // extern "C"
