// Host runtime behind the C ABI declared in include/ibm_lbm.h: handle state,
// carving of the caller's device buffers, validation, the per-step kernel
// sequence (Sec. II.C sub-steps 1-5), hipGraph replay, profiling and errors.
#include <algorithm>
#include <cmath>
#include <mutex>
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

// HIP events of a profiling or tuning call, destroyed when the call returns,
// also on its early error returns.
struct EventPool {
  std::vector<hipEvent_t> v;
  hipError_t make(hipEvent_t *e) {
    v.push_back(nullptr);
    hipError_t r = hipEventCreate(&v.back());
    *e = v.back();
    return r;
  }
  ~EventPool() {
    for (hipEvent_t e : v)
      if (e) (void)hipEventDestroy(e);
  }
};

// Steps replayed per graph launch (even, so that the buffer parity returns).
constexpr int GRAPH_STEPS = 16;

struct LatticeLayout {
  long long N, S;
  int gsh;             // log2 of the rows per population group
  int nxs;             // population row stride (nx rounded up to a multiple of 4)
  int tpr;             // lanes per row of the row-form kernels (0: not used)
  long long pop_elems;  // elements of one population buffer
  int tnx, tny, tnz;
  size_t off_ctrl, off_stamp[2], off_nstamp, off_U, off_g[2], off_f[2], total;
};

LatticeLayout lattice_layout(int nx, int ny, int nz, int storage) {
  LatticeLayout l{};
  l.N = (long long)nx * ny * nz;
  l.S = (long long)round_up((size_t)l.N, 64);
  const ibm::PopGeometry pg = ibm::pop_geometry(nx, ny, nz);
  l.nxs = pg.nxs;
  l.gsh = pg.gsh;
  l.pop_elems = pg.pop_elems;
  l.tpr = pg.tpr;
  l.tnx = (nx + ibm::TILE_X - 1) / ibm::TILE_X;
  l.tny = (ny + ibm::TILE_Y - 1) / ibm::TILE_Y;
  l.tnz = (nz + ibm::TILE_Z - 1) / ibm::TILE_Z;
  const size_t tiles = (size_t)l.tnx * l.tny * l.tnz;
  const size_t es = (storage & IBM_STORAGE_FP16) ? 2 : 4;
  const int nbuf = (storage & IBM_STORAGE_ONE_BUFFER) ? 1 : 2;
  size_t off = 0;
  l.off_ctrl = off;
  off += round_up(sizeof(ibm::Ctrl), ALIGN);
  for (int k = 0; k < 2; ++k) {
    l.off_stamp[k] = off;
    off += round_up(tiles * sizeof(int), ALIGN);
  }
  l.off_nstamp = off;
  off += round_up((size_t)l.S * sizeof(int), ALIGN);
  l.off_U = off;
  off += round_up((size_t)l.S * 16, ALIGN);
  for (int k = 0; k < 2; ++k) {
    l.off_g[k] = off;
    off += round_up(3 * (size_t)l.S * sizeof(float), ALIGN);
  }
  for (int k = 0; k < 2; ++k) {
    l.off_f[k] = k < nbuf ? off : l.off_f[0];  // one buffer: both names, one array
    if (k < nbuf) off += round_up((size_t)l.pop_elems * es, ALIGN);
  }
  l.total = off;
  return l;
}

struct MembraneLayout {
  size_t x, u, F, ext_id, node_cap, csr_off, csr_ent, tri, ref_p, ref_ghi, ref_glo, origin, moduli,
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
  int nx = 0, ny = 0, nz = 0, storage = 0;  // storage: IBM_STORAGE_FP32 or IBM_STORAGE_FP16
  bool one_buffer = false;                  // IBM_STORAGE_ONE_BUFFER: the AA pattern only
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
  std::vector<int> csr_off, csr_ent;  // host copy of the node -> (face, corner) lists

  // default collide-stream form: whole-row vectors where the row fits a
  // wavefront, else two nodes per thread, non-temporal, 128-thread blocks;
  // cached row stores for population buffers of CACHED_POP_MIN..MAX bytes
  int use_graph = 1, eq_linear = 0, ab2 = 0, recenter_every = 64, lbm_variant = 16 | 7;
  int box_mode = 0;     // IBM_OPT_STENCIL_BOX: bit 0 box spreading, bit 1 / bit 2
                        // interpolation through LDS boxes / the node-velocity field
  bool box_set = false;  // box_mode chosen by the caller (else set with the membrane)
  bool have_prev_u = false;
  int64_t since_recenter = 0;

  // 16-step graphs, one per parity of the step count at which they start
  // (the buffer each step reads is fixed in the captured launches)
  hipGraphExec_t gexec[2] = {nullptr, nullptr};

  // IBM_OPT_OVERLAP: the lattice update of graph-replayed steps split into the
  // force slab L.zlo <= z < L.zhi and the rest, which rides along with the
  // coupling kernels
  int overlap = 0;
  bool slab_stale = true;  // the slab must be measured again before the next graph

  bool has_tan = false;  // a tangent (forward sensitivity) state is attached
  ibm::TanDev T{};
};

namespace {

// A population buffer of this many bytes: the row form stores the new
// populations with ordinary (cached) writes by default, so that the buffer the
// next step reads largely stays in the 256 MB last-level cache.  Measured per
// buffer size: 80-160 MB steps 4-14 % faster (128^3 FP32 and FP16, the dense
// suspension in FP16); 254-319 MB 1-14 % slower (the dense suspension in FP32,
// the batched sweep); 20 MB (64^3 FP32) 12 % slower, 2.5 MB 2 % faster.
constexpr long long CACHED_POP_MIN = 48LL << 20, CACHED_POP_MAX = 192LL << 20;

// IBM_OPT_LBM_VARIANT and the device rows of its bit 8 (all rows)
void set_variant(ibm_lattice *lat, int v) {
  lat->lbm_variant = v;
  lat->L.cached_rows = (v & 256) ? lat->ny * lat->nz : 0;
}

void invalidate_graph(ibm_lattice *lat) {
  for (hipGraphExec_t &g : lat->gexec) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  lat->slab_stale = true;
}

// Clear the tile stamps and both force fields (they hold nothing between
// steps that the next step needs: its spreading writes its own field).
void clear_force_fields(ibm_lattice *lat, hipStream_t s) {
  const long long tiles = (long long)lat->lay.tnx * lat->lay.tny * lat->lay.tnz;
  for (int k = 0; k < 2; ++k) {
    ibm::launch_fill_u32(lat->L.stamp[k], tiles, (uint32_t)(-100), s);
    ibm::launch_fill_u32(lat->L.g[k], 3 * lat->lay.S, 0u, s);
  }
  ibm::launch_fill_u32(lat->L.nstamp, lat->lay.S, (uint32_t)(-100), s);
}

// Clear the control words, the tile stamps and both force fields.
void reset_force_state(ibm_lattice *lat, hipStream_t s) {
  ibm::launch_fill_u32(lat->base + lat->lay.off_ctrl, sizeof(ibm::Ctrl) / 4, 0u, s);
  clear_force_fields(lat, s);
}

// Interpolation mode of the coupling kernels (launch_interp_advect) for an
// IBM_OPT_STENCIL_BOX value: bit 2 (the node-velocity field) over bit 1 (LDS
// boxes) over the per-stencil-node evaluation.
int interp_mode(int box_mode) { return (box_mode & 4) ? 2 : ((box_mode & 2) ? 1 : 0); }

// Population state after `steps` completed steps, as the readers take it
// (pop_buffer and pop_swapped, stored_post): two buffers, the buffer steps & 1; the AA pattern,
// buffer 0 after an even number of steps and the swapped state 2 after an odd
// number.
int pop_state(const ibm_lattice *lat, int64_t steps) {
  if (lat->L.aa) return (steps & 1) ? 2 : 0;
  return (int)(steps & 1);
}

// Enqueue one full timestep on stream s (Sec. II.C, sub-steps 1-5).
void enqueue_step(ibm_lattice *lat, hipStream_t s, int advect) {
  const int src = (int)(lat->steps & 1);
  const int par = src;  // force field of this step's parity
  const bool tan = lat->has_tan;
  if (lat->has_mem) {
    ibm::launch_spread(lat->L, lat->M, par, lat->box_mode & 1, s);       // 1, 2: F(t), f(X, t)
    if (tan) ibm::launch_tangent_spread(lat->L, lat->M, lat->T, par, s);
    ibm::launch_collide_stream(lat->L, lat->storage, src, par, true,     // 3: f_i(t+1)
                               lat->eq_linear != 0, lat->lbm_variant, s);
    if (tan) {
      ibm::launch_tangent_collide_stream(lat->L, lat->T, src, par, lat->eq_linear != 0, s);
      // before the positions move: the tangent needs x(t)
      ibm::launch_tangent_interp(lat->L, lat->M, lat->T, src ^ 1, par, s);
    }
    ibm::launch_interp_advect(lat->L, lat->M, lat->storage,              // 4, 5
                              pop_state(lat, lat->steps + 1), par, advect,
                              interp_mode(lat->box_mode), s);
  } else {
    ibm::launch_collide_stream(lat->L, lat->storage, src, par, false, lat->eq_linear != 0,
                               lat->lbm_variant, s);
    if (tan) ibm::launch_tangent_collide_stream(lat->L, lat->T, src, par, lat->eq_linear != 0, s);
  }
  lat->steps += 1;
  lat->since_recenter += 1;
}

int advect_mode(ibm_lattice *lat) { return (lat->ab2 && lat->have_prev_u) ? 1 : 0; }

bool split_update(const ibm_lattice *lat) {
  return lat->L.zlo > 0 || lat->L.zhi < lat->nz || lat->L.ylo > 0 || lat->L.yhi < lat->ny;
}

// IBM_OPT_OVERLAP: measure the membranes' extent (waits) and set the force
// slab of rows zlo <= z < zhi (all y): stencils reach 1 below and 2 above a
// node's floor(z); the margin covers the drift until the next re-centring;
// the slab is rounded out to the 4^3 force tiles.  The whole lattice when the
// option is off or not applicable (no row form, a tangent), or when
// the slab holds more than three quarters of the rows.  (The slab spans all
// y: rows updated inside the coupling launches cost more than in the
// lattice kernel, as the coupling kernels' dependent loads then wait behind
// their traffic, so a narrower box in y measured slower.)
int refresh_slab(ibm_lattice *lat) {
  int zlo = 0, zhi = lat->nz, ylo = 0, yhi = lat->ny;
  if (lat->overlap && lat->has_mem && !lat->has_tan && lat->L.tpr > 0 && !lat->L.aa) {
    ibm::launch_node_range(lat->M, lat->L.ctrl, lat->stream);
    int r[4] = {0, 0, 0, 0};  // zmin, zmax, ymin, ymax
    IBM_HIP(hipMemcpyAsync(r, &lat->L.ctrl->zmin, sizeof(r), hipMemcpyDeviceToHost, lat->stream));
    IBM_HIP(hipStreamSynchronize(lat->stream));
    const int margin = 4 + (int)std::ceil(2.0 * std::fabs(lat->uw) * lat->recenter_every);
    const int za = r[0] - 1 - margin, zb = r[1] + 3 + margin;
    zlo = za <= 0 ? 0 : za / 4 * 4;
    zhi = zb >= lat->nz ? lat->nz : std::min(lat->nz, (zb + 3) / 4 * 4);
    // value 1: only where at least 2^20 nodes lie outside the slab (below that
    // the fixed costs of the split outweigh the overlap: measured slower on
    // 64^3 with half the rows outside); value 2: wherever the slab applies
    const long long outside = (long long)(lat->nz - (zhi - zlo)) * lat->ny * lat->nx;
    if (4LL * (zhi - zlo) > 3LL * lat->nz || (lat->overlap == 1 && outside < (1LL << 20))) {
      zlo = ylo = 0;
      zhi = lat->nz;
      yhi = lat->ny;
    }
  }
  ibm::LatDev &L = lat->L;
  if (zlo != L.zlo || zhi != L.zhi || ylo != L.ylo || yhi != L.yhi) {
    L.zlo = zlo;
    L.zhi = zhi;
    L.ylo = ylo;
    L.yhi = yhi;
    invalidate_graph(lat);
    // Rows outside a slab take the force-free update, which neither reads
    // nor clears the force field.  A tile the last step stamped outside the
    // new slab would keep its force under that stamp, and a later spreading
    // into it would add onto it: start the fields afresh.
    clear_force_fields(lat, lat->stream);
  }
  lat->slab_stale = false;
  return IBM_OK;
}

// Graph steps with the lattice update split at the force slab (rows with z in
// [zlo, zhi); the row sets also take a box in y, here the whole lattice): the
// other rows need no force.  Those above the slab ride along with the
// spreading of the same step, those below it with the interpolation of the
// step before (a step's update only needs that step's populations), so only
// the slab waits for the spreading.  The first step's
// rows of the second kind go first on their own; the last interpolation
// carries no rows (the next step is not begun).
void enqueue_steps_split(ibm_lattice *lat, hipStream_t s, int nsteps, int advect) {
  const ibm::LatDev &L = lat->L;
  const bool linear = lat->eq_linear != 0;
  const int mode = interp_mode(lat->box_mode);
  const int slab = L.zhi - L.zlo;
  const ibm::RowSet near{0, 0, L.zlo, L.ylo, L.yhi - L.ylo, slab * (L.yhi - L.ylo)};
  const ibm::RowSet low{0, L.zlo * L.ny, L.zlo, 0, std::max(1, L.ylo), slab * L.ylo};
  const ibm::RowSet high{L.zhi * L.ny, (L.nz - L.zhi) * L.ny, L.zlo, L.yhi, std::max(1, L.ny - L.yhi),
                         slab * (L.ny - L.yhi)};
  const ibm::RowSet none{0, 0, 0, 0, 1, 0};
  const int src0 = (int)(lat->steps & 1);
  ibm::launch_collide_stream_rows(L, lat->storage, src0, src0, false, linear, low, s);
  for (int k = 0; k < nsteps; ++k) {
    const int src = (int)(lat->steps & 1);
    const int par = src;
    ibm::launch_spread_far(L, lat->M, par, lat->box_mode & 1, lat->storage, linear, src, high, s);
    ibm::launch_collide_stream_rows(L, lat->storage, src, par, true, linear, near, s);
    ibm::launch_interp_far(L, lat->M, lat->storage, src ^ 1, par, advect, mode, linear,
                           k + 1 < nsteps ? low : none, s);
    lat->steps += 1;
    lat->since_recenter += 1;
  }
}

// Capture the graph for the current parity of the step count.
int capture_graph(ibm_lattice *lat) {
  const int p = (int)(lat->steps & 1);
  if (lat->gexec[p]) (void)hipGraphExecDestroy(lat->gexec[p]);
  lat->gexec[p] = nullptr;
  if (!lat->cap_stream) IBM_HIP(hipStreamCreateWithFlags(&lat->cap_stream, hipStreamNonBlocking));
  const int64_t saved_steps = lat->steps, saved_since = lat->since_recenter;
  hipGraph_t graph = nullptr;
  IBM_HIP(hipStreamBeginCapture(lat->cap_stream, hipStreamCaptureModeThreadLocal));
  if (split_update(lat)) {
    enqueue_steps_split(lat, lat->cap_stream, GRAPH_STEPS, advect_mode(lat));
  } else {
    for (int k = 0; k < GRAPH_STEPS; ++k) enqueue_step(lat, lat->cap_stream, advect_mode(lat));
  }
  hipError_t e = hipStreamEndCapture(lat->cap_stream, &graph);
  lat->steps = saved_steps;
  lat->since_recenter = saved_since;
  if (e != hipSuccess) return fail(IBM_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&lat->gexec[p], graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    lat->gexec[p] = nullptr;
    return fail(IBM_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
  }
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
    // after a stencil outside the split update's slab, the slab is measured
    // again from the nodes' current extent before the next step
    if (err & ibm::ERR_SLAB) lat->slab_stale = true;
    if (err & ibm::ERR_WALL)
      return fail(IBM_ERR_STENCIL_HITS_WALL, "a delta stencil reached beyond a wall");
    if (err & ibm::ERR_FACE)
      return fail(IBM_ERR_INVERTED_FACE, "a membrane face degenerated (det C <= 0)");
    if (err & ibm::ERR_NONFINITE) return fail(IBM_ERR_NONFINITE, "non-finite observables");
    if (err & ibm::ERR_SLAB)
      return fail(IBM_ERR_OUTSIDE_SLAB, "a stencil reached outside the force slab of the split update");
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

// Order of a capsule's nodes by recursive coordinate bisection: the set is
// cut across its longest extent, at the multiple of PATCH (in the membrane's
// global node numbering, the capsule starting at node `base`) nearest to its
// middle, until a set lies within one run of PATCH global node numbers; each
// such patch is then taken in Morton order.  So every run of PATCH
// consecutive nodes from a multiple of PATCH (the nodes of one spreading
// block, or of 4 or 8 blocks for the wider deltas) holds one compact patch of
// the surface, except where one capsule ends and the next begins, and a
// block's stencils span a small box.  A Morton curve alone sometimes joins
// two distant pieces of the surface in one such run.
constexpr int PATCH = 32;

void bisect_order(const double *xyz, int *idx, int n, int base, std::vector<int> &out) {
  const int first = base / PATCH * PATCH + PATCH;  // first patch boundary after base
  if (base + n <= first) {
    std::vector<double> sub(3 * (size_t)n);
    for (int k = 0; k < n; ++k)
      for (int d = 0; d < 3; ++d) sub[3 * (size_t)k + d] = xyz[3 * (size_t)idx[k] + d];
    const std::vector<int> o = morton_order(sub.data(), n);
    for (int k = 0; k < n; ++k) out.push_back(idx[o[k]]);
    return;
  }
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int k = 0; k < n; ++k)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], xyz[3 * (size_t)idx[k] + d]);
      hi[d] = std::max(hi[d], xyz[3 * (size_t)idx[k] + d]);
    }
  int axis = 0;
  for (int d = 1; d < 3; ++d)
    if (hi[d] - lo[d] > hi[axis] - lo[axis]) axis = d;
  // the patch boundary inside (base, base + n) nearest to the middle
  const int last = (base + n - 1) / PATCH * PATCH;  // last boundary before the end
  int cut = (base + n / 2 + PATCH / 2) / PATCH * PATCH;
  cut = std::max(first, std::min(cut, last));
  const int left = cut - base;
  std::nth_element(idx, idx + left, idx + n, [&](int a, int b) {
    const double xa = xyz[3 * (size_t)a + axis], xb = xyz[3 * (size_t)b + axis];
    return xa < xb || (xa == xb && a < b);
  });
  bisect_order(xyz, idx, left, base, out);
  bisect_order(xyz, idx + left, n - left, cut, out);
}

std::vector<int> patch_order(const double *xyz, int n, int base) {
  std::vector<int> idx(n), out;
  out.reserve(n);
  for (int k = 0; k < n; ++k) idx[k] = k;
  bisect_order(xyz, idx.data(), n, base, out);
  return out;
}

}  // namespace

struct ibm_batch {
  std::vector<ibm_lattice *> runs;
  hipStream_t stream = nullptr;      // the first run's stream
  hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
  char *dev = nullptr;
  size_t bytes = 0;
  size_t cap_lat = 0, cap_node = 0;  // work-item capacities
  ibm::BatchDev B{};
  std::vector<char> image;  // host copy of the device tables last uploaded
  // 16-step graphs per parity of the step count, and the options each was
  // captured with
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  int graph_advect[2] = {-1, -1}, graph_linear[2] = {-1, -1};
  int box_mode = 0;  // default stencil-box mode of the batched coupling kernels
  // ibm_batch_autotune's choices: stencil-box mode per delta width (index m,
  // -1: box_mode), wavefronts per block of the row-form lattice update, and
  // the fraction 1 / cached_div of each run's rows stored with cached writes
  // (0: none)
  int class_mode[5] = {-1, -1, -1, -1, -1};
  int wpb = 4, cached_div = 4;
  int persistent = 0;  // one cooperative launch per step instead of graphs of
                       // per-phase launches (where every run uses the row form)
};

namespace {

struct BatchLayout {
  size_t lat, mem, lat_items, node_items, total;
};

BatchLayout batch_layout(size_t n, size_t cap_lat, size_t cap_node) {
  BatchLayout l{};
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t at = off;
    off += round_up(b, ALIGN);
    return at;
  };
  l.lat = take(n * sizeof(ibm::LatDev));
  l.mem = take(n * sizeof(ibm::MemDev));
  l.lat_items = take(cap_lat * sizeof(int2));
  l.node_items = take(cap_node * sizeof(int2));
  l.total = off;
  return l;
}

long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }

// Lanes per membrane node in the batched coupling kernels.
int group_lanes(int m) { return ibm::batch_group_size(m); }

// Work items of the batched kernels for the runs' current state, with wpb
// wavefronts per block of the lattice update (batch_lat_blocks).
void batch_items(const std::vector<ibm_lattice *> &runs, int wpb, std::vector<int2> &li,
                 std::vector<int2> &ni) {
  li.clear();
  ni.clear();
  for (size_t r = 0; r < runs.size(); ++r) {
    const ibm_lattice *lat = runs[r];
    const long long nb = ibm::batch_lat_blocks(lat->L, wpb);
    for (long long b = 0; b < nb; ++b) li.push_back(make_int2((int)r, (int)b));
    if (!lat->has_mem) continue;
    const long long nbn = ceil_div((long long)lat->M.nn * group_lanes(lat->M.m), 256);
    for (long long b = 0; b < nbn; ++b) ni.push_back(make_int2((int)r, (int)b));
  }
}

// Whether the runs with capsules hold the node velocities of a previous step
// (needed by Adams-Bashforth advection).
bool batch_prev_u(const ibm_batch *b) {
  for (const ibm_lattice *lat : b->runs)
    if (lat->has_mem) return lat->have_prev_u;
  return false;
}

void batch_invalidate_graph(ibm_batch *b) {
  for (hipGraphExec_t &g : b->gexec) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
}

// Check that the runs can step together and bring the device tables up to
// date with their current state (a run's membrane or options may have
// changed since the last batch step).
int batch_sync_tables(ibm_batch *b) {
  const ibm_lattice *r0 = b->runs[0];
  for (const ibm_lattice *lat : b->runs) {
    if (lat->steps != r0->steps)
      return fail(IBM_ERR_BAD_STATE, "batched runs must have made the same number of steps");
    if (lat->storage != r0->storage || lat->eq_linear != r0->eq_linear || lat->ab2 != r0->ab2)
      return fail(IBM_ERR_BAD_STATE,
                  "batched runs need the same storage, equilibrium and advection options");
    if (lat->stream != r0->stream)
      return fail(IBM_ERR_BAD_STATE, "batched runs must share one stream");
    if (lat->has_tan) return fail(IBM_ERR_BAD_STATE, "batched runs cannot carry a tangent");
    if (lat->L.aa) return fail(IBM_ERR_BAD_STATE, "batched runs use two population buffers");
    if (lat->has_mem && lat->have_prev_u != batch_prev_u(b))
      return fail(IBM_ERR_BAD_STATE, "batched runs differ in their stored node velocities");
  }
  std::vector<int2> li, ni;
  batch_items(b->runs, b->wpb, li, ni);
  if (li.size() > b->cap_lat || ni.size() > b->cap_node)
    return fail(IBM_ERR_BAD_STATE, "the runs' membranes grew since the batch was created");
  // the first run's explicit choice, else box spreading and interpolation
  // from the node-velocity field once the whole batch makes at least 256
  // blocks of coupling work; ibm_batch_autotune's per-width choices first
  b->box_mode = r0->box_set ? r0->box_mode : (ni.size() >= 256 ? 1 | 4 : 0);
  bool any_field = false;
  const size_t n = b->runs.size();
  const BatchLayout bl = batch_layout(n, b->cap_lat, b->cap_node);
  std::vector<char> img(bl.total, 0);
  for (size_t r = 0; r < n; ++r) {
    ibm::LatDev Lr = b->runs[r]->L;  // batches update the whole lattice
    // the runs together outgrow the last-level cache: only the first quarter
    // of each run's rows is stored cached (measured on the 64-run sweep:
    // +4.6 % FP32, +2.4 % FP16; half or all of the rows: slower)
    Lr.cached_rows = b->cached_div ? Lr.ny * Lr.nz / b->cached_div : 0;
    Lr.zlo = Lr.ylo = 0;
    Lr.zhi = Lr.nz;
    Lr.yhi = Lr.ny;
    std::memcpy(img.data() + bl.lat + r * sizeof(ibm::LatDev), &Lr, sizeof(ibm::LatDev));
    ibm::MemDev Mr = b->runs[r]->M;
    const int cm = b->runs[r]->has_mem ? b->class_mode[Mr.m] : -1;
    Mr.cmode = cm >= 0 ? cm : b->box_mode;
    any_field = any_field || (b->runs[r]->has_mem && (Mr.cmode & 4));
    std::memcpy(img.data() + bl.mem + r * sizeof(ibm::MemDev), &Mr, sizeof(ibm::MemDev));
  }
  std::memcpy(img.data() + bl.lat_items, li.data(), li.size() * sizeof(int2));
  std::memcpy(img.data() + bl.node_items, ni.data(), ni.size() * sizeof(int2));
  ibm::BatchDev B{};
  B.lat = reinterpret_cast<const ibm::LatDev *>(b->dev + bl.lat);
  B.mem = reinterpret_cast<const ibm::MemDev *>(b->dev + bl.mem);
  B.lat_items = reinterpret_cast<const int2 *>(b->dev + bl.lat_items);
  B.node_items = reinterpret_cast<const int2 *>(b->dev + bl.node_items);
  B.n_lat_items = (int)li.size();
  B.n_node_items = (int)ni.size();
  B.wpb = b->wpb;
  B.any_field = any_field ? 1 : 0;
  const bool same = img == b->image && std::memcmp(&B, &b->B, sizeof(B)) == 0;
  if (!same) {
    IBM_HIP(hipMemcpyAsync(b->dev, img.data(), img.size(), hipMemcpyHostToDevice, b->stream));
    IBM_HIP(hipStreamSynchronize(b->stream));  // img must outlive the copy
    b->image.swap(img);
    b->B = B;
    batch_invalidate_graph(b);
  }
  return IBM_OK;
}

// Enqueue one timestep of every run (Sec. II.C, sub-steps 1-5), one launch
// per kernel.
void enqueue_batch_step(ibm_batch *b, hipStream_t s, int advect) {
  const ibm_lattice *r0 = b->runs[0];
  const int src = (int)(r0->steps & 1), par = src;
  ibm::launch_batch_spread(b->B, par, s);
  ibm::launch_batch_collide_stream(b->B, r0->storage, src, par, r0->eq_linear != 0, s);
  ibm::launch_batch_interp(b->B, r0->storage, src ^ 1, par, advect, s);
  for (ibm_lattice *lat : b->runs) {
    lat->steps += 1;
    lat->since_recenter += 1;
  }
}

int batch_capture_graph(ibm_batch *b, int advect) {
  const int p = (int)(b->runs[0]->steps & 1);
  if (b->gexec[p]) (void)hipGraphExecDestroy(b->gexec[p]);
  b->gexec[p] = nullptr;
  if (!b->cap_stream) IBM_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  std::vector<int64_t> steps, since;
  for (ibm_lattice *lat : b->runs) {
    steps.push_back(lat->steps);
    since.push_back(lat->since_recenter);
  }
  hipGraph_t graph = nullptr;
  IBM_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < GRAPH_STEPS; ++k) enqueue_batch_step(b, b->cap_stream, advect);
  hipError_t e = hipStreamEndCapture(b->cap_stream, &graph);
  for (size_t r = 0; r < b->runs.size(); ++r) {
    b->runs[r]->steps = steps[r];
    b->runs[r]->since_recenter = since[r];
  }
  if (e != hipSuccess) return fail(IBM_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&b->gexec[p], graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    b->gexec[p] = nullptr;
    return fail(IBM_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
  }
  b->graph_advect[p] = advect;
  b->graph_linear[p] = b->runs[0]->eq_linear;
  return IBM_OK;
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
  if (storage & ~(IBM_STORAGE_FP16 | IBM_STORAGE_ONE_BUFFER))
    return fail(IBM_ERR_INVALID_ARG, "unknown storage %d", storage);
  if ((storage & IBM_STORAGE_ONE_BUFFER) && (nx % 4 || ibm::pop_geometry(nx, ny, nz).tpr <= 0))
    return fail(IBM_ERR_INVALID_ARG,
                "one population buffer (the AA pattern) needs nx a multiple of 4 and at most 256");
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
  lat->one_buffer = (storage & IBM_STORAGE_ONE_BUFFER) != 0;
  storage &= IBM_STORAGE_FP16;  // lat->storage: the precision
  lat->storage = storage;
  lat->tau = tau;
  lat->stream = static_cast<hipStream_t>(stream);
  lat->base = static_cast<char *>(dev_state);
  lat->lay = lattice_layout(nx, ny, nz, storage | (lat->one_buffer ? IBM_STORAGE_ONE_BUFFER : 0));
  ibm::LatDev &L = lat->L;
  L.nx = nx;
  L.ny = ny;
  L.nz = nz;
  L.tnx = lat->lay.tnx;
  L.tny = lat->lay.tny;
  L.tnz = lat->lay.tnz;
  L.S = lat->lay.S;
  L.gsh = lat->lay.gsh;
  L.nxs = lat->lay.nxs;
  L.tpr = lat->lay.tpr;
  L.rpw = L.tpr ? 64 / L.tpr : 0;
  {
    const long long pb = lat->lay.pop_elems * (storage == IBM_STORAGE_FP16 ? 2 : 4);
    set_variant(lat, lat->lbm_variant | (pb >= CACHED_POP_MIN && pb <= CACHED_POP_MAX ? 256 : 0));
  }
  for (int i = 0; i < ibm::Q; ++i) L.pst[i] = (long long)i * ((long long)L.nxs << L.gsh);
  for (int k = 0; k < 2; ++k) {
    L.f[k] = lat->base + lat->lay.off_f[k];
    L.g[k] = reinterpret_cast<float *>(lat->base + lat->lay.off_g[k]);
    L.stamp[k] = reinterpret_cast<int *>(lat->base + lat->lay.off_stamp[k]);
  }
  L.ctrl = reinterpret_cast<ibm::Ctrl *>(lat->base + lat->lay.off_ctrl);
  L.nstamp = reinterpret_cast<int *>(lat->base + lat->lay.off_nstamp);
  L.U = reinterpret_cast<float4 *>(lat->base + lat->lay.off_U);
  L.inv_tau = (float)(1.0 / tau);
  L.guo_pre = (float)(1.0 - 0.5 / tau);
  L.uw = 0.0f;
  L.aa = lat->one_buffer ? 1 : 0;
  L.mass_fix = 0;
  L.zlo = 0;
  L.zhi = nz;
  L.ylo = 0;
  L.yhi = ny;
  for (int i = 0; i < ibm::Q; ++i) L.h_scale[i] = L.h_inv[i] = 1.0f;
  if (storage == IBM_STORAGE_FP16) {
    // Deviations f_i - w_i scaled by 2^k / w_i keep a shear-flow population
    // (|f_i - w_i| <~ 0.1 w_i) in FP16's normal range with 11 significant bits.
    for (int i = 0; i < ibm::Q; ++i) {
      L.h_scale[i] = (float)(16.0 / ibm::wgt(i));
      L.h_inv[i] = 1.0f / L.h_scale[i];
    }
  }
  reset_force_state(lat, lat->stream);
  for (int k = 0; k < (lat->one_buffer ? 1 : 2); ++k) {
    const size_t words = ((size_t)lat->lay.pop_elems * (storage == IBM_STORAGE_FP16 ? 2 : 4) + 3) / 4;
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
  if (lat->has_tan) return fail(IBM_ERR_BAD_STATE, "detach the tangent before adding a membrane");
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

  // internal node order: each capsule's nodes in compact patches (patch_order)
  std::vector<int> ext_of_int(nn), int_of_ext(nn);
  for (int c = 0; c < n_caps; ++c) {
    const int n0 = node_off[c];
    const std::vector<int> order = patch_order(xyz + 3 * (size_t)n0, nodes_per_cap[c], n0);
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
  lat->csr_off = csr_off;
  lat->csr_ent = csr_ent;
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
  ibm::launch_reference_geometry(M, lat->L.ctrl, s);
  IBM_HIP(hipGetLastError());
  IBM_HIP(hipStreamSynchronize(s));  // host vectors must outlive the copies
  lat->has_mem = true;
  rc = check_device(lat);
  if (rc) {
    lat->has_mem = false;
    return rc;
  }
  // Box spreading pays once there are enough blocks for atomic conflicts
  // between overlapping stencils to dominate (measured: 256+ blocks); box
  // interpolation on such membranes too, now that each block's nodes form a
  // compact patch (measured: 128^3 +1.3 %, the dense suspension +2.2 %).
  // Where the stencil nodes number at least an eighth of the lattice nodes,
  // interpolation reads the node-velocity field instead (one pass evaluates
  // each touched node once): the dense suspension's step 1.5 % faster; on
  // 128^3 with one capsule (stencils on 8 % of the nodes) 5 % slower, the
  // pass scanning the whole lattice for few marks.
  if (!lat->box_set) {
    const int gs = m == 2 ? ibm::group_size<2>() : (m == 3 ? ibm::group_size<3>() : ibm::group_size<4>());
    const long long stencil_nodes = (long long)nn * m * m * m;
    const long long lattice_nodes = (long long)lat->nx * lat->ny * lat->nz;
    lat->box_mode = (long long)nn * gs >= 256LL * 256 ? (8 * stencil_nodes >= lattice_nodes ? 5 : 3) : 0;
  }
  // the force bookkeeping restarts with the membrane
  reset_force_state(lat, s);
  lat->have_prev_u = false;
  lat->since_recenter = 0;
  invalidate_graph(lat);
  IBM_HIP(hipStreamSynchronize(s));
  return ok();
}

int ibm_split_box(ibm_lattice *lat, int *box) {
  if (!lat || !box) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  if (lat->slab_stale && (lat->overlap || split_update(lat))) {
    int rc = refresh_slab(lat);
    if (rc) return rc;
  }
  box[0] = lat->L.zlo;
  box[1] = lat->L.zhi;
  box[2] = lat->L.ylo;
  box[3] = lat->L.yhi;
  return ok();
}

int ibm_step(ibm_lattice *lat, int64_t n) {
  if (!lat) return fail(IBM_ERR_INVALID_ARG, "lat is NULL");
  if (n < 0) return fail(IBM_ERR_INVALID_ARG, "negative step count");
  if (lat->has_tan && lat->ab2)
    return fail(IBM_ERR_BAD_STATE, "the tangent model follows Euler advection only");
  while (n > 0) {
    const bool want_graph = lat->use_graph && n >= GRAPH_STEPS && (!lat->ab2 || lat->have_prev_u);
    // Re-centre when due, or early when the next graph would run past the
    // interval (re-centring only changes the frame, so earlier is harmless):
    // every graph launch then fits.
    if (lat->has_mem && (lat->since_recenter >= lat->recenter_every ||
                         (want_graph && lat->since_recenter > 0 &&
                          lat->since_recenter + GRAPH_STEPS > lat->recenter_every))) {
      ibm::launch_recenter(lat->M, lat->stream);
      lat->since_recenter = 0;
      if (lat->overlap) lat->slab_stale = true;
    }
    if (lat->slab_stale && (lat->overlap || split_update(lat))) {
      int rc = refresh_slab(lat);
      if (rc) return rc;
    }
    const bool graph_ok =
        want_graph && (!lat->has_mem || lat->since_recenter + GRAPH_STEPS <= lat->recenter_every);
    if (graph_ok) {
      const int p = (int)(lat->steps & 1);
      if (!lat->gexec[p]) {
        int rc = capture_graph(lat);
        if (rc) return rc;
      }
      IBM_HIP(hipGraphLaunch(lat->gexec[p], lat->stream));
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
  const int src = pop_state(lat, lat->steps);
  const int gpar = (lat->has_mem && lat->steps > 0) ? (int)((lat->steps - 1) & 1) : -1;
  ibm::launch_get_field(lat->L, lat->storage, src, gpar, what, dst_dev, lat->stream);
  IBM_HIP(hipGetLastError());
  int rc = check_device(lat);
  return rc ? rc : ok();
}

int ibm_set_fields(ibm_lattice *lat, int what, const double *src_dev) {
  if (!lat || !src_dev) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  if (what != IBM_FIELD_POPS) return fail(IBM_ERR_INVALID_ARG, "only the populations can be set");
  if (lat->L.aa && (lat->steps & 1))
    return fail(IBM_ERR_BAD_STATE,
                "with the AA pattern the populations can be set after an even number of steps only");
  ibm::launch_set_pops(lat->L, lat->storage, lat->L.aa ? 0 : (int)(lat->steps & 1), src_dev,
                       lat->stream);
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
  lat->slab_stale = true;  // the nodes moved: the force slab is measured again
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

int ibm_deformation_gradient(ibm_lattice *lat, int capsule, double *grad_dev) {
  if (!lat || !grad_dev) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  if (!lat->has_mem) return fail(IBM_ERR_BAD_STATE, "no membrane attached");
  if (capsule < 0 || capsule >= lat->M.n_caps)
    return fail(IBM_ERR_INVALID_ARG, "capsule %d out of range", capsule);
  ibm::launch_obs_grad64(lat->M, capsule, grad_dev, lat->stream);
  IBM_HIP(hipGetLastError());
  int rc = check_device(lat);
  return rc ? rc : ok();
}

int ibm_totals_bytes(const ibm_lattice *lat, size_t *bytes) {
  if (!lat || !bytes) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  *bytes = (size_t)ibm::totals_parts(lat->L) * sizeof(double4);
  return ok();
}

int ibm_lattice_totals(ibm_lattice *lat, void *work_dev, size_t work_bytes, double *out_dev) {
  if (!lat || !work_dev || !out_dev) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  const size_t need = (size_t)ibm::totals_parts(lat->L) * sizeof(double4);
  if (work_bytes < need)
    return fail(IBM_ERR_INVALID_ARG, "work_dev has %zu bytes, %zu needed", work_bytes, need);
  if (((uintptr_t)work_dev) % 32 || ((uintptr_t)out_dev) % 8)
    return fail(IBM_ERR_INVALID_ARG, "work_dev must be 32-byte and out_dev 8-byte aligned");
  ibm::launch_totals(lat->L, lat->storage, pop_state(lat, lat->steps), static_cast<double4 *>(work_dev),
                     out_dev, lat->stream);
  IBM_HIP(hipGetLastError());
  return ok();
}

}  // extern "C"

// Partial sums of ibm_lattice_totals_noalloc: a file-scope device array, one
// copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel or a copy (on the host it is only a stand-in for
// the symbol): it uses the device address that hipGetSymbolAddress gives for
// the current device, taken once per device and kept in noalloc_ptr.
constexpr int NOALLOC_PARTS = 8192;  // lattices of up to 8192 * 4096 nodes
static __device__ __align__(256) double4 scratch[NOALLOC_PARTS];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mu;
double4 *noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// The scratch address on the device that owns the lattice's stream (that
// device made current while the symbol is looked up).
int noalloc_scratch(hipStream_t stream, double4 **out) {
  int dev = -1, cur = -1;
  IBM_HIP(hipStreamGetDevice(stream, &dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return fail(IBM_ERR_BAD_STATE, "device %d beyond the %d the library keeps scratch for", dev,
                NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> g(noalloc_mu);
  if (!noalloc_ptr[dev]) {
    IBM_HIP(hipGetDevice(&cur));
    if (cur != dev) IBM_HIP(hipSetDevice(dev));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) IBM_HIP(hipSetDevice(cur));
    if (e != hipSuccess)
      return fail(IBM_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    noalloc_ptr[dev] = static_cast<double4 *>(p);
  }
  *out = noalloc_ptr[dev];
  return IBM_OK;
}

}  // namespace

extern "C" {

int ibm_lattice_totals_noalloc(ibm_lattice *lat, double *out_dev) {
  if (!lat || !out_dev) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  if (((uintptr_t)out_dev) % 8) return fail(IBM_ERR_INVALID_ARG, "out_dev must be 8-byte aligned");
  const int np = ibm::totals_parts(lat->L);
  if (np > NOALLOC_PARTS)
    return fail(IBM_ERR_INVALID_ARG,
                "a lattice of %lld nodes needs %d partial sums; the built-in scratch holds %d "
                "(lattices of up to %lld nodes): use ibm_lattice_totals with a workspace",
                (long long)lat->nx * lat->ny * lat->nz, np, NOALLOC_PARTS,
                (long long)NOALLOC_PARTS * ibm::TOTALS_NODES);
  double4 *part = nullptr;
  int rc = noalloc_scratch(lat->stream, &part);
  if (rc) return rc;
  // every partial the final pass reads is written first by this call, so
  // nothing needs clearing
  ibm::launch_totals(lat->L, lat->storage, pop_state(lat, lat->steps), part, out_dev, lat->stream);
  IBM_HIP(hipGetLastError());
  return ok();
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
      if (value < 0 || value > 511) return fail(IBM_ERR_INVALID_ARG, "variant is 0..511");
      set_variant(lat, value);
      break;
    case IBM_OPT_OVERLAP:
      if (value < 0 || value > 2) return fail(IBM_ERR_INVALID_ARG, "overlap is 0, 1 or 2");
      lat->overlap = value;
      invalidate_graph(lat);
      break;
    case IBM_OPT_STREAMING:
      if (value != IBM_STREAM_TWO_BUFFERS && value != IBM_STREAM_AA)
        return fail(IBM_ERR_INVALID_ARG, "streaming is 0 (two buffers) or 1 (AA)");
      if (value == IBM_STREAM_AA && (lat->L.tpr <= 0 || lat->nx % 4 || lat->has_tan))
        return fail(IBM_ERR_BAD_STATE,
                    "the AA pattern needs rows of at most 256 nodes, nx a multiple of 4 and no tangent");
      if (lat->one_buffer && value != IBM_STREAM_AA)
        return fail(IBM_ERR_BAD_STATE, "a lattice with one population buffer streams with the AA pattern");
      if (value != lat->L.aa && (lat->steps & 1))
        return fail(IBM_ERR_BAD_STATE, "the streaming pattern changes after an even number of steps only");
      lat->L.aa = value;
      // the split update has no AA form: back to the whole lattice at once
      if (value && split_update(lat)) {
        int rc = refresh_slab(lat);
        if (rc) return rc;
      }
      break;
    case IBM_OPT_FP16_MASS:
      if (value != 0 && value != 1) return fail(IBM_ERR_INVALID_ARG, "FP16 mass correction is 0 or 1");
      if (value && (lat->storage != IBM_STORAGE_FP16 || lat->L.tpr <= 0))
        return fail(IBM_ERR_BAD_STATE,
                    "the FP16 mass correction needs FP16 storage and the row form (nx <= 256)");
      lat->L.mass_fix = value;
      break;
    case IBM_OPT_STENCIL_BOX:
      if (value < 0 || value > 7) return fail(IBM_ERR_INVALID_ARG, "stencil box mode is 0..7");
      lat->box_mode = value;
      lat->box_set = true;
      break;
    default:
      return fail(IBM_ERR_INVALID_ARG, "unknown option %d", option);
  }
  invalidate_graph(lat);
  return ok();
}

int ibm_autotune(ibm_lattice *lat, int steps_per_trial, int *chosen) {
  if (!lat) return fail(IBM_ERR_INVALID_ARG, "lat is NULL");
  if (steps_per_trial < GRAPH_STEPS || steps_per_trial > 65536)
    return fail(IBM_ERR_INVALID_ARG, "steps_per_trial must be in %d..65536", GRAPH_STEPS);
  const int n = (steps_per_trial + GRAPH_STEPS - 1) / GRAPH_STEPS * GRAPH_STEPS;
  EventPool pool;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  IBM_HIP(pool.make(&e0));
  IBM_HIP(pool.make(&e1));
  int rc = IBM_OK;
  // the better of two timings of n steps, after a settling graph replay
  auto trial = [&](float &ms) -> int {
    int r = ibm_step(lat, GRAPH_STEPS);
    if (r) return r;
    ms = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      IBM_HIP(hipEventRecord(e0, lat->stream));
      r = ibm_step(lat, n);
      if (r) return r;
      IBM_HIP(hipEventRecord(e1, lat->stream));
      IBM_HIP(hipEventSynchronize(e1));
      float t = 0.0f;
      IBM_HIP(hipEventElapsedTime(&t, e0, e1));
      ms = std::min(ms, t);
    }
    return check_device(lat);
  };
  if (lat->steps & 1) rc = ibm_step(lat, 1);
  if (!rc) rc = ibm_step(lat, 4 * n);  // clocks and caches settle before the first trial
  // collide-stream form: the row-vector kernel where rows fit, and the
  // per-node kernel with or without two nodes per thread, non-temporal
  // accesses, 256- or 128-thread blocks
  std::vector<int> cand;
  const bool rows_ok = lat->L.tpr > 0;
  if (rows_ok) {
    cand.push_back(16);
    cand.push_back(16 | 256);
  }
  for (int nt : {2, 0})
    for (int v2 : {1, 0})
      for (int thr : {4, 0})
        if (!(v2 && lat->nx % 2)) cand.push_back(nt | v2 | thr);
  int best_v = lat->lbm_variant, best_b = lat->box_mode;
  float best = 1e30f;
  for (int v : cand) {
    if (rc) break;
    set_variant(lat, v);
    invalidate_graph(lat);
    float ms = 0.0f;
    rc = trial(ms);
    if (!rc && ms < best) {
      best = ms;
      best_v = v;
    }
  }
  set_variant(lat, best_v);
  invalidate_graph(lat);
  if (!rc && lat->has_mem) {
    best = 1e30f;
    for (int bm = 0; bm < 6 && !rc; ++bm) {  // 6, 7 interpolate as 4, 5
      lat->box_mode = bm;
      invalidate_graph(lat);
      float ms = 0.0f;
      rc = trial(ms);
      if (!rc && ms < best) {
        best = ms;
        best_b = bm;
      }
    }
    lat->box_mode = best_b;
    lat->box_set = true;
    invalidate_graph(lat);
  }
  if (!rc && lat->has_mem && !lat->has_tan && lat->L.tpr > 0) {
    // the split lattice update, where its slab leaves enough rows outside
    float ms_off = 0.0f, ms_on = 0.0f;
    lat->overlap = 0;
    invalidate_graph(lat);
    rc = trial(ms_off);
    if (!rc) {
      lat->overlap = 1;
      invalidate_graph(lat);
      rc = trial(ms_on);
    }
    lat->overlap = (!rc && split_update(lat) && ms_on < ms_off) ? 1 : 0;  // 1 can fall back
    invalidate_graph(lat);
  }
  if (rc) return rc;
  if (chosen) {
    chosen[0] = lat->lbm_variant;
    chosen[1] = lat->box_mode;
  }
  return ok();
}

// Plain (not captured) steps with marker events around each phase; with
// kernel_ms, the lattice-update kernel of every step also records its own
// dispatch's start and end, and *kernel_ms receives their mean difference.
static int profile_steps(ibm_lattice *lat, int64_t n, double *ms_per_phase, double *kernel_ms) {
  if (lat->has_tan) return fail(IBM_ERR_BAD_STATE, "detach the tangent before profiling");
  if (n < 1 || n > 4096) return fail(IBM_ERR_INVALID_ARG, "profile 1..4096 steps");
  const int ne = lat->has_mem ? 5 : 2;
  EventPool pool;
  std::vector<hipEvent_t> ev((size_t)n * ne);
  std::vector<ibm::DispatchTimer> kt(kernel_ms ? (size_t)n : 0);
  for (auto &e : ev) IBM_HIP(pool.make(&e));
  for (auto &t : kt) {
    IBM_HIP(pool.make(&t.start));
    IBM_HIP(pool.make(&t.stop));
  }
  hipStream_t s = lat->stream;
  for (int64_t k = 0; k < n; ++k) {
    if (lat->has_mem && lat->since_recenter >= lat->recenter_every) {
      ibm::launch_recenter(lat->M, s);
      lat->since_recenter = 0;
      if (lat->overlap) lat->slab_stale = true;
    }
    hipEvent_t *e = &ev[(size_t)k * ne];
    const ibm::DispatchTimer *t = kernel_ms ? &kt[(size_t)k] : nullptr;
    const int src = (int)(lat->steps & 1), par = src;
    IBM_HIP(hipEventRecord(e[0], s));
    if (lat->has_mem) {
      IBM_HIP(hipEventRecord(e[1], s));  // the forces are formed by the spreading kernel
      ibm::launch_spread(lat->L, lat->M, par, lat->box_mode & 1, s);
      IBM_HIP(hipEventRecord(e[2], s));
      ibm::launch_collide_stream(lat->L, lat->storage, src, par, true, lat->eq_linear != 0,
                                 lat->lbm_variant, s, 0, -1, t);
      IBM_HIP(hipEventRecord(e[3], s));
      ibm::launch_interp_advect(lat->L, lat->M, lat->storage, pop_state(lat, lat->steps + 1), par,
                                advect_mode(lat), interp_mode(lat->box_mode), s);
      IBM_HIP(hipEventRecord(e[4], s));
      if (lat->ab2) lat->have_prev_u = true;
    } else {
      ibm::launch_collide_stream(lat->L, lat->storage, src, par, false, lat->eq_linear != 0,
                                 lat->lbm_variant, s, 0, -1, t);
      IBM_HIP(hipEventRecord(e[1], s));
    }
    lat->steps += 1;
    lat->since_recenter += 1;
  }
  IBM_HIP(hipGetLastError());
  IBM_HIP(hipStreamSynchronize(s));
  double acc[IBM_N_PHASES] = {0.0, 0.0, 0.0, 0.0}, kacc = 0.0;
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
    if (kernel_ms) {
      IBM_HIP(hipEventElapsedTime(&ms, kt[(size_t)k].start, kt[(size_t)k].stop));
      kacc += ms;
    }
  }
  if (ms_per_phase)
    for (int p = 0; p < IBM_N_PHASES; ++p) ms_per_phase[p] = acc[p] / (double)n;
  if (kernel_ms) *kernel_ms = kacc / (double)n;
  int rc = check_device(lat);
  return rc ? rc : ok();
}

int ibm_profile_step(ibm_lattice *lat, int64_t n, double *ms_per_phase) {
  if (!lat || !ms_per_phase) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  return profile_steps(lat, n, ms_per_phase, nullptr);
}

int ibm_profile_lattice_kernel(ibm_lattice *lat, int64_t n, double *ms) {
  if (!lat || !ms) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  return profile_steps(lat, n, nullptr, ms);
}

int ibm_destroy(ibm_lattice *lat) {
  if (!lat) return ok();
  (void)hipStreamSynchronize(lat->stream);
  invalidate_graph(lat);
  if (lat->cap_stream) (void)hipStreamDestroy(lat->cap_stream);
  delete lat;
  return ok();
}

// ---- tangent (forward sensitivity) --------------------------------------------------
namespace {
struct TangentLayout {
  size_t df[2], dg[2], dx, du, dF, dmod, obs, total;
};

TangentLayout tangent_layout(const ibm_lattice *lat) {
  TangentLayout l{};
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t at = off;
    off += round_up(b, ALIGN);
    return at;
  };
  const size_t S = (size_t)lat->lay.S;
  const size_t nn = lat->has_mem ? (size_t)lat->M.nn : 0, nc = lat->has_mem ? (size_t)lat->M.n_caps : 0;
  for (int k = 0; k < 2; ++k) l.df[k] = take(ibm::Q * S * sizeof(float));
  for (int k = 0; k < 2; ++k) l.dg[k] = take(3 * S * sizeof(float));
  l.dx = take(nn * 16);
  l.du = take(nn * 16);
  l.dF = take(nn * 16);
  l.dmod = take(nc * 8);
  l.obs = take(2 * nc * IBM_OBS_N * sizeof(double));
  l.total = off;
  return l;
}
}  // namespace

int ibm_tangent_bytes(ibm_lattice *lat, size_t *bytes) {
  if (!lat || !bytes) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  if (lat->one_buffer) return fail(IBM_ERR_BAD_STATE, "the tangent model needs two population buffers");
  *bytes = tangent_layout(lat).total;
  return ok();
}

int ibm_tangent_attach(ibm_lattice *lat, const double *dks, const double *dka, double duw,
                       int init_profile, void *dev_mem, size_t bytes) {
  if (!lat) return fail(IBM_ERR_INVALID_ARG, "lat is NULL");
  if (lat->storage != IBM_STORAGE_FP32)
    return fail(IBM_ERR_BAD_STATE, "the tangent model needs FP32 population storage");
  if (lat->L.aa) return fail(IBM_ERR_BAD_STATE, "the tangent model needs two population buffers");
  if (lat->has_mem && (!dks || !dka)) return fail(IBM_ERR_INVALID_ARG, "dks and dka are needed");
  if (!std::isfinite(duw)) return fail(IBM_ERR_INVALID_ARG, "duw must be finite");
  const TangentLayout tl = tangent_layout(lat);
  if (!dev_mem || ((uintptr_t)dev_mem) % ALIGN)
    return fail(IBM_ERR_INVALID_ARG, "dev_mem NULL or not 256-byte aligned");
  if (bytes < tl.total) return fail(IBM_ERR_INVALID_ARG, "dev_mem has %zu bytes, %zu needed", bytes, tl.total);
  char *b = static_cast<char *>(dev_mem);
  ibm::TanDev T{};
  for (int k = 0; k < 2; ++k) {
    T.df[k] = reinterpret_cast<float *>(b + tl.df[k]);
    T.dg[k] = reinterpret_cast<float *>(b + tl.dg[k]);
  }
  T.dx = reinterpret_cast<float4 *>(b + tl.dx);
  T.du = reinterpret_cast<float4 *>(b + tl.du);
  T.dF = reinterpret_cast<float4 *>(b + tl.dF);
  T.dmod = reinterpret_cast<float2 *>(b + tl.dmod);
  T.obs = reinterpret_cast<double *>(b + tl.obs);
  T.duw = (float)duw;
  hipStream_t s = lat->stream;
  std::vector<float2> dm;
  if (lat->has_mem) {
    for (int c = 0; c < lat->M.n_caps; ++c) {
      if (!std::isfinite(dks[c]) || !std::isfinite(dka[c]))
        return fail(IBM_ERR_INVALID_ARG, "capsule %d: non-finite modulus rate", c);
      dm.push_back(make_float2((float)dks[c], (float)dka[c]));
    }
    IBM_HIP(hipMemcpyAsync(T.dmod, dm.data(), dm.size() * sizeof(float2), hipMemcpyHostToDevice, s));
    for (float4 *p : {T.dx, T.du, T.dF}) ibm::launch_fill_u32(p, 4LL * lat->M.nn, 0u, s);
  }
  for (int k = 0; k < 2; ++k) {
    ibm::launch_fill_u32(T.dg[k], 3 * lat->lay.S, 0u, s);
    ibm::launch_fill_u32(T.df[k], (long long)ibm::Q * lat->lay.S, 0u, s);
  }
  ibm::launch_tangent_init(lat->L, T, (int)(lat->steps & 1), init_profile ? 1 : 0,
                           lat->eq_linear, s);
  IBM_HIP(hipGetLastError());
  IBM_HIP(hipStreamSynchronize(s));  // dm must outlive the copy
  lat->T = T;
  lat->has_tan = true;
  invalidate_graph(lat);
  return ok();
}

int ibm_tangent_detach(ibm_lattice *lat) {
  if (!lat) return fail(IBM_ERR_INVALID_ARG, "lat is NULL");
  IBM_HIP(hipStreamSynchronize(lat->stream));
  lat->has_tan = false;
  lat->T = ibm::TanDev{};
  invalidate_graph(lat);
  return ok();
}

int ibm_tangent_get_pops(ibm_lattice *lat, double *dst_dev) {
  if (!lat || !dst_dev) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  if (!lat->has_tan) return fail(IBM_ERR_BAD_STATE, "no tangent attached");
  ibm::launch_get_tangent_pops(lat->L, lat->T, (int)(lat->steps & 1), dst_dev, lat->stream);
  IBM_HIP(hipGetLastError());
  int rc = check_device(lat);
  return rc ? rc : ok();
}

int ibm_tangent_get_mesh(ibm_lattice *lat, double *dxyz_dev, double *du_dev) {
  if (!lat) return fail(IBM_ERR_INVALID_ARG, "lat is NULL");
  if (!lat->has_tan || !lat->has_mem) return fail(IBM_ERR_BAD_STATE, "no tangent membrane state");
  ibm::MemDev M2 = lat->M;  // the mesh readout, pointed at the tangent arrays
  M2.F = lat->T.dx;
  M2.u = lat->T.du;
  ibm::launch_get_mesh(M2, nullptr, dxyz_dev, du_dev, lat->stream);
  IBM_HIP(hipGetLastError());
  int rc = check_device(lat);
  return rc ? rc : ok();
}

int ibm_tangent_observables(ibm_lattice *lat, double h, double *out_host) {
  if (!lat || !out_host) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  if (!lat->has_tan || !lat->has_mem) return fail(IBM_ERR_BAD_STATE, "no tangent membrane state");
  if (!(h > 0.0) || !std::isfinite(h)) return fail(IBM_ERR_INVALID_ARG, "h must be > 0");
  const size_t k = (size_t)lat->M.n_caps * IBM_OBS_N;
  ibm::launch_observables_shifted(lat->M, lat->L.ctrl, lat->T.dx, h, lat->T.obs, lat->stream);
  ibm::launch_observables_shifted(lat->M, lat->L.ctrl, lat->T.dx, -h, lat->T.obs + k, lat->stream);
  IBM_HIP(hipGetLastError());
  std::vector<double> both(2 * k);
  IBM_HIP(hipMemcpyAsync(both.data(), lat->T.obs, 2 * k * sizeof(double), hipMemcpyDeviceToHost,
                         lat->stream));
  int rc = check_device(lat);
  if (rc) return rc;
  for (size_t q = 0; q < k; ++q) out_host[q] = (both[q] - both[k + q]) / (2.0 * h);
  return ok();
}

// ---- adjoint (reverse-mode gradient) -------------------------------------------
namespace {
struct AdjointLayout {
  long long n_ck, pop;
  size_t ck_f, ck_x, seg_f, seg_x, lf[2], lU, lg, lx, lx_tmp, lF, pk, uw_col, stamp, part, total;
};

AdjointLayout adjoint_layout(const ibm_lattice *lat, int64_t steps, int K) {
  AdjointLayout l{};
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t at = off;
    off += round_up(b, ALIGN);
    return at;
  };
  const size_t pop = (size_t)lat->lay.pop_elems, S = (size_t)lat->lay.S, nn = (size_t)lat->M.nn;
  l.pop = (long long)pop;
  l.n_ck = (steps + K - 1) / K + 1;  // every K steps from 0, and the final state
  l.ck_f = take((size_t)l.n_ck * pop * 4);
  l.ck_x = take((size_t)l.n_ck * nn * 16);
  l.seg_f = take(((size_t)K + 1) * pop * 4);
  l.seg_x = take((size_t)K * nn * 16);
  for (int k = 0; k < 2; ++k) l.lf[k] = take(pop * 4);
  l.lU = take(3 * S * 4);
  l.lg = take(3 * S * 4);
  l.lx = take(nn * 16);
  l.lx_tmp = take(nn * 16);
  l.lF = take(nn * 16);
  l.pk = take(nn * 16);
  l.uw_col = take(2 * (size_t)lat->nx * lat->ny * 8);
  l.stamp = take((size_t)lat->lay.tnx * lat->lay.tny * lat->lay.tnz * 4);
  l.part = take((size_t)ibm::adj_couette_blocks(lat->L) * 8);
  l.total = off;
  return l;
}

hipError_t copy_d2d(void *dst, const void *src, size_t bytes, hipStream_t s) {
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
}

// Force fields cleared, tiles unstamped, device step counter set.
void adjoint_reset_fields(ibm_lattice *lat, uint32_t step, hipStream_t s) {
  const long long tiles = (long long)lat->lay.tnx * lat->lay.tny * lat->lay.tnz;
  for (int k = 0; k < 2; ++k) {
    ibm::launch_fill_u32(lat->L.stamp[k], tiles, (uint32_t)(-100), s);
    ibm::launch_fill_u32(lat->L.g[k], 3 * lat->lay.S, 0u, s);
  }
  ibm::launch_fill_u32(&lat->L.ctrl->step, 1, step, s);
}
}  // namespace

int ibm_adjoint_bytes(ibm_lattice *lat, int64_t steps, int checkpoint_every, size_t *bytes) {
  if (!lat || !bytes) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  if (!lat->has_mem) return fail(IBM_ERR_BAD_STATE, "no membrane attached");
  if (steps < 1 || checkpoint_every < 1) return fail(IBM_ERR_INVALID_ARG, "steps and checkpoint_every must be >= 1");
  if (lat->one_buffer) return fail(IBM_ERR_BAD_STATE, "the adjoint needs two population buffers");
  *bytes = adjoint_layout(lat, steps, checkpoint_every).total;
  return ok();
}

int ibm_adjoint_gradient(ibm_lattice *lat, int64_t steps, int checkpoint_every, int capsule,
                         int couette_start, void *dev_mem, size_t bytes, double *D_out,
                         double *dD_dks, double *dD_dka, double *dD_duw) {
  if (!lat || !dev_mem || !D_out || !dD_dks || !dD_dka || !dD_duw)
    return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  if (!lat->has_mem) return fail(IBM_ERR_BAD_STATE, "no membrane attached");
  if (lat->storage != IBM_STORAGE_FP32) return fail(IBM_ERR_BAD_STATE, "the adjoint needs FP32 storage");
  if (lat->L.aa) return fail(IBM_ERR_BAD_STATE, "the adjoint needs two population buffers");
  if (lat->ab2) return fail(IBM_ERR_BAD_STATE, "the adjoint follows Euler advection only");
  if (lat->has_tan) return fail(IBM_ERR_BAD_STATE, "detach the tangent first");
  if (capsule < 0 || capsule >= lat->M.n_caps) return fail(IBM_ERR_INVALID_ARG, "no capsule %d", capsule);
  if (steps < 1 || checkpoint_every < 1)
    return fail(IBM_ERR_INVALID_ARG, "steps and checkpoint_every must be >= 1");
  const int K = checkpoint_every;
  const AdjointLayout al = adjoint_layout(lat, steps, K);
  if (((uintptr_t)dev_mem) % ALIGN) return fail(IBM_ERR_INVALID_ARG, "dev_mem not 256-byte aligned");
  if (bytes < al.total) return fail(IBM_ERR_INVALID_ARG, "dev_mem has %zu bytes, %zu needed", bytes, al.total);
  int rc = check_device(lat);
  if (rc) return rc;
  hipStream_t s = lat->stream;
  char *b = static_cast<char *>(dev_mem);
  ibm::MemDev &M = lat->M;
  const size_t pop_bytes = (size_t)al.pop * 4, x_bytes = (size_t)M.nn * 16;
  auto ck_f = [&](long long k) { return b + al.ck_f + (size_t)k * pop_bytes; };
  auto ck_x = [&](long long k) { return b + al.ck_x + (size_t)k * x_bytes; };
  auto seg_f = [&](long long k) { return reinterpret_cast<float *>(b + al.seg_f + (size_t)k * pop_bytes); };
  auto seg_x = [&](long long k) { return b + al.seg_x + (size_t)k * x_bytes; };
  ibm::AdjDev A{};
  for (int k = 0; k < 2; ++k) A.lf[k] = reinterpret_cast<float *>(b + al.lf[k]);
  A.lU = reinterpret_cast<float *>(b + al.lU);
  A.lg = reinterpret_cast<float *>(b + al.lg);
  A.lx = reinterpret_cast<float4 *>(b + al.lx);
  A.lx_tmp = reinterpret_cast<float4 *>(b + al.lx_tmp);
  A.lF = reinterpret_cast<float4 *>(b + al.lF);
  A.pk = reinterpret_cast<double2 *>(b + al.pk);
  A.uw_col = reinterpret_cast<double *>(b + al.uw_col);
  A.stamp = reinterpret_cast<int *>(b + al.stamp);
  double *part = reinterpret_cast<double *>(b + al.part);

  int c0 = 0;  // the device step counter the stamps refer to
  IBM_HIP(hipMemcpy(&c0, &lat->L.ctrl->step, sizeof(int), hipMemcpyDeviceToHost));
  const int64_t s0 = lat->steps;
  // fixed frames: the reverse pass replays the same steps; restored on every exit
  struct RecenterGuard {
    ibm_lattice *lat;
    int saved;
    ~RecenterGuard() {
      lat->recenter_every = saved;
      lat->since_recenter = 0;
      invalidate_graph(lat);
    }
  } guard{lat, lat->recenter_every};
  lat->recenter_every = 0x7fffffff;
  invalidate_graph(lat);
  auto fbuf = [&](int64_t t) { return lat->L.f[(s0 + t) & 1]; };
  const bool linear = lat->eq_linear != 0;

  // forward pass with checkpoints
  for (int64_t t = 0; t < steps; ++t) {
    if (t % K == 0) {
      IBM_HIP(copy_d2d(ck_f(t / K), fbuf(t), pop_bytes, s));
      IBM_HIP(copy_d2d(ck_x(t / K), M.x, x_bytes, s));
    }
    enqueue_step(lat, s, 0);
  }
  IBM_HIP(copy_d2d(ck_f(al.n_ck - 1), fbuf(steps), pop_bytes, s));
  IBM_HIP(copy_d2d(ck_x(al.n_ck - 1), M.x, x_bytes, s));

  // objective D(T) of the capsule and its gradient with respect to x(T)
  ibm::launch_observables(M, lat->L.ctrl, s);
  for (void *p : {(void *)A.lx, (void *)A.pk}) ibm::launch_fill_u32(p, 4LL * M.nn, 0u, s);
  ibm::launch_obs_grad(M, capsule, A.lx, s);
  for (int k = 0; k < 2; ++k) ibm::launch_fill_u32(A.lf[k], al.pop, 0u, s);
  ibm::launch_fill_u32(A.lU, 3 * lat->lay.S, 0u, s);
  ibm::launch_fill_u32(A.lg, 3 * lat->lay.S, 0u, s);
  ibm::launch_fill_u32(A.uw_col, 4LL * lat->nx * lat->ny, 0u, s);
  ibm::launch_fill_u32(A.stamp, (long long)lat->lay.tnx * lat->lay.tny * lat->lay.tnz,
                       (uint32_t)(-100), s);

  // reverse pass, segment by segment: recompute and store the segment's
  // states from its checkpoint, then reverse its steps
  int cur = 0;  // A.lf[cur] holds the adjoint of f(t + 1)
  const long long nseg = (steps + K - 1) / K;
  for (long long seg = nseg - 1; seg >= 0; --seg) {
    const int64_t sb = seg * K, se = std::min<int64_t>(sb + K, steps);
    lat->steps = s0 + sb;
    IBM_HIP(copy_d2d(fbuf(sb), ck_f(seg), pop_bytes, s));
    IBM_HIP(copy_d2d(M.x, ck_x(seg), x_bytes, s));
    adjoint_reset_fields(lat, (uint32_t)(c0 + sb), s);
    for (int64_t t = sb; t < se; ++t) {
      IBM_HIP(copy_d2d(seg_f(t - sb), fbuf(t), pop_bytes, s));
      IBM_HIP(copy_d2d(seg_x(t - sb), M.x, x_bytes, s));
      enqueue_step(lat, s, 0);
    }
    IBM_HIP(copy_d2d(seg_f(se - sb), fbuf(se), pop_bytes, s));
    for (int64_t t = se - 1; t >= sb; --t) {
      const int par = (int)((s0 + t) & 1);
      const int step = (int)(c0 + t);
      IBM_HIP(copy_d2d(M.x, seg_x(t - sb), x_bytes, s));
      ibm::launch_fill_u32(&lat->L.ctrl->step, 1, (uint32_t)step, s);
      ibm::launch_fill_u32(lat->L.g[par], 3 * lat->lay.S, 0u, s);
      ibm::launch_spread(lat->L, M, par, lat->box_mode & 1, s);  // F(t), g(t)
      const float *f0 = seg_f(t - sb), *f1 = seg_f(t + 1 - sb);
      ibm::launch_adj_interp(lat->L, M, A, f1, par, step, s);
      ibm::launch_adj_velocity(lat->L, A, f1, par, step, cur, s);
      ibm::launch_adj_collide_stream(lat->L, A, f0, par, step, cur, linear, s);
      ibm::launch_adj_spread(lat->L, M, A, s);
      ibm::launch_adj_fem(lat->L, M, A, s);
      cur ^= 1;
    }
  }
  const long long nparts = couette_start ? ibm::adj_couette_blocks(lat->L) : 0;
  if (couette_start) ibm::launch_adj_couette_start(lat->L, A, cur, linear ? 1 : 0, part, s);

  // back to the forward state at the end of the run
  lat->steps = s0 + steps;
  IBM_HIP(copy_d2d(fbuf(steps), ck_f(al.n_ck - 1), pop_bytes, s));
  IBM_HIP(copy_d2d(M.x, ck_x(al.n_ck - 1), x_bytes, s));
  adjoint_reset_fields(lat, (uint32_t)(c0 + steps), s);
  lat->have_prev_u = false;
  IBM_HIP(hipGetLastError());

  std::vector<double2> pk(M.nn);
  std::vector<double> uw(2 * (size_t)lat->nx * lat->ny), parts((size_t)nparts);
  std::vector<double> obs((size_t)M.n_caps * IBM_OBS_N);
  IBM_HIP(hipMemcpyAsync(pk.data(), A.pk, pk.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
  IBM_HIP(hipMemcpyAsync(uw.data(), A.uw_col, uw.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  if (nparts) IBM_HIP(hipMemcpyAsync(parts.data(), part, parts.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  IBM_HIP(hipMemcpyAsync(obs.data(), M.obs, obs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  rc = check_device(lat);
  if (rc) return rc;
  for (int c = 0; c < M.n_caps; ++c) {
    double a = 0.0, k = 0.0;
    for (int n = lat->node_off[c]; n < lat->node_off[c + 1]; ++n) {
      a += pk[n].x;
      k += pk[n].y;
    }
    dD_dks[c] = a;
    dD_dka[c] = k;
  }
  double du = 0.0;
  for (double v : uw) du += v;
  for (double v : parts) du += v;
  *dD_duw = du;
  *D_out = obs[(size_t)capsule * IBM_OBS_N + IBM_OBS_D];
  return ok();
}

int ibm_batch_bytes(int n_runs, ibm_lattice *const *runs, size_t *bytes) {
  if (n_runs < 1 || !runs || !bytes) return fail(IBM_ERR_INVALID_ARG, "need n_runs >= 1 and runs");
  for (int r = 0; r < n_runs; ++r) {
    if (!runs[r]) return fail(IBM_ERR_INVALID_ARG, "run %d is NULL", r);
    if (runs[r]->one_buffer) return fail(IBM_ERR_BAD_STATE, "batched runs use two population buffers");
  }
  std::vector<ibm_lattice *> v(runs, runs + n_runs);
  std::vector<int2> li, ni;
  batch_items(v, 1, li, ni);  // the most lattice items: one wavefront per block
  *bytes = batch_layout(v.size(), li.size(), ni.size()).total;
  return ok();
}

int ibm_batch_create(int n_runs, ibm_lattice *const *runs, void *dev_mem, size_t bytes,
                     ibm_batch **out) {
  if (!out) return fail(IBM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  int rc = ibm_batch_bytes(n_runs, runs, &need);
  if (rc) return rc;
  if (!dev_mem || ((uintptr_t)dev_mem) % ALIGN)
    return fail(IBM_ERR_INVALID_ARG, "dev_mem NULL or not 256-byte aligned");
  if (bytes < need) return fail(IBM_ERR_INVALID_ARG, "dev_mem has %zu bytes, %zu needed", bytes, need);
  std::vector<ibm_lattice *> v(runs, runs + n_runs);
  for (int r = 0; r < n_runs; ++r)
    for (int q = 0; q < r; ++q)
      if (v[q] == v[r]) return fail(IBM_ERR_INVALID_ARG, "run %d appears twice", r);
  std::vector<int2> li, ni;
  batch_items(v, 1, li, ni);
  ibm_batch *b = new ibm_batch();
  b->runs = v;
  b->stream = v[0]->stream;
  b->dev = static_cast<char *>(dev_mem);
  b->bytes = bytes;
  b->cap_lat = li.size();
  b->cap_node = ni.size();
  rc = batch_sync_tables(b);
  if (rc) {
    delete b;
    return rc;
  }
  *out = b;
  return ok();
}

int ibm_batch_step(ibm_batch *b, int64_t n) {
  if (!b) return fail(IBM_ERR_INVALID_ARG, "batch is NULL");
  if (n < 0) return fail(IBM_ERR_INVALID_ARG, "negative step count");
  int rc = batch_sync_tables(b);
  if (rc) return rc;
  ibm_lattice *r0 = b->runs[0];
  bool rows_only = true;
  for (const ibm_lattice *lat : b->runs) rows_only = rows_only && lat->L.tpr > 0;
  while (n > 0 && b->persistent && rows_only) {
    for (ibm_lattice *lat : b->runs)
      if (lat->has_mem && lat->since_recenter >= lat->recenter_every) {
        ibm::launch_recenter(lat->M, b->stream);
        lat->since_recenter = 0;
        if (lat->overlap) lat->slab_stale = true;
      }
    const int src = (int)(r0->steps & 1);
    const int advect = (r0->ab2 && batch_prev_u(b)) ? 1 : 0;
    if (ibm::launch_batch_persistent(b->B, r0->storage, src, src, advect, r0->eq_linear != 0,
                                     b->stream))
      return fail(IBM_ERR_HIP, "the persistent batched step could not be launched: %s",
                  hipGetErrorString(hipGetLastError()));
    for (ibm_lattice *lat : b->runs) {
      lat->steps += 1;
      lat->since_recenter += 1;
      if (lat->ab2 && lat->has_mem) lat->have_prev_u = true;
    }
    n -= 1;
  }
  while (n > 0) {
    const bool prev = batch_prev_u(b);
    const bool want_graph = n >= GRAPH_STEPS && (!r0->ab2 || prev);
    bool room = true;
    for (ibm_lattice *lat : b->runs) {
      // due, or early so that the next graph fits (as in ibm_step)
      if (lat->has_mem && (lat->since_recenter >= lat->recenter_every ||
                           (want_graph && lat->since_recenter > 0 &&
                            lat->since_recenter + GRAPH_STEPS > lat->recenter_every))) {
        ibm::launch_recenter(lat->M, b->stream);
        lat->since_recenter = 0;
        if (lat->overlap) lat->slab_stale = true;  // for the run's own later steps
      }
      if (lat->has_mem && lat->since_recenter + GRAPH_STEPS > lat->recenter_every) room = false;
    }
    const int advect = (r0->ab2 && prev) ? 1 : 0;
    const bool graph_ok = want_graph && room;
    if (graph_ok) {
      const int p = (int)(r0->steps & 1);
      if (!b->gexec[p] || b->graph_advect[p] != advect || b->graph_linear[p] != r0->eq_linear) {
        rc = batch_capture_graph(b, advect);
        if (rc) return rc;
      }
      IBM_HIP(hipGraphLaunch(b->gexec[p], b->stream));
      for (ibm_lattice *lat : b->runs) {
        lat->steps += GRAPH_STEPS;
        lat->since_recenter += GRAPH_STEPS;
      }
      n -= GRAPH_STEPS;
    } else {
      enqueue_batch_step(b, b->stream, advect);
      if (r0->ab2)
        for (ibm_lattice *lat : b->runs)
          if (lat->has_mem) lat->have_prev_u = true;
      n -= 1;
    }
  }
  IBM_HIP(hipGetLastError());
  return ok();
}

int ibm_batch_set_persistent(ibm_batch *b, int on) {
  if (!b) return fail(IBM_ERR_INVALID_ARG, "batch is NULL");
  if (on != 0 && on != 1) return fail(IBM_ERR_INVALID_ARG, "persistent is 0 or 1");
  b->persistent = on;
  return ok();
}

int ibm_batch_autotune(ibm_batch *b, int steps_per_trial, int *chosen) {
  if (!b) return fail(IBM_ERR_INVALID_ARG, "batch is NULL");
  if (steps_per_trial < GRAPH_STEPS || steps_per_trial > 65536)
    return fail(IBM_ERR_INVALID_ARG, "steps_per_trial must be in %d..65536", GRAPH_STEPS);
  const int n = (steps_per_trial + GRAPH_STEPS - 1) / GRAPH_STEPS * GRAPH_STEPS;
  EventPool pool;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  IBM_HIP(pool.make(&e0));
  IBM_HIP(pool.make(&e1));
  // the better of two timings of n steps, after the graphs of the candidate
  // are captured and replayed once
  auto trial = [&](float &ms) -> int {
    batch_invalidate_graph(b);
    int r = ibm_batch_step(b, GRAPH_STEPS);
    if (!r) r = ibm_batch_step(b, 1);
    if (!r) r = ibm_batch_step(b, GRAPH_STEPS);
    if (r) return r;
    ms = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      IBM_HIP(hipEventRecord(e0, b->stream));
      r = ibm_batch_step(b, n);
      if (r) return r;
      IBM_HIP(hipEventRecord(e1, b->stream));
      IBM_HIP(hipEventSynchronize(e1));
      float t = 0.0f;
      IBM_HIP(hipEventElapsedTime(&t, e0, e1));
      ms = std::min(ms, t);
    }
    for (ibm_lattice *lat : b->runs) {
      r = check_device(lat);
      if (r) return r;
    }
    return IBM_OK;
  };
  int rc = ibm_batch_step(b, 4 * n);  // clocks and caches settle before the first trial
  // 1. the row-form block shape and the fraction of rows stored cached
  int best_w = b->wpb, best_c = b->cached_div;
  float best = 1e30f;
  for (int w : {4, 2, 1})
    for (int cd : {4, 2, 0}) {
      if (rc) break;
      b->wpb = w;
      b->cached_div = cd;
      float ms = 0.0f;
      rc = trial(ms);
      if (!rc && ms < best) {
        best = ms;
        best_w = w;
        best_c = cd;
      }
    }
  b->wpb = best_w;
  b->cached_div = best_c;
  // 2. the stencil-box mode of each delta width present, one width at a time
  bool present[5] = {false, false, false, false, false};
  for (const ibm_lattice *lat : b->runs)
    if (lat->has_mem) present[lat->M.m] = true;
  for (int m = 2; m <= 4 && !rc; ++m) {
    if (!present[m]) continue;
    int best_m = b->class_mode[m];
    best = 1e30f;
    for (int mode : {0, 1, 3, 5}) {
      b->class_mode[m] = mode;
      float ms = 0.0f;
      rc = trial(ms);
      if (rc) break;
      if (ms < best) {
        best = ms;
        best_m = mode;
      }
    }
    b->class_mode[m] = best_m;
  }
  // 3. one persistent launch per step against the graphs of per-phase launches
  if (!rc) {
    bool rows_only = true;
    for (const ibm_lattice *lat : b->runs) rows_only = rows_only && lat->L.tpr > 0;
    if (rows_only) {
      float ms_graph = 0.0f, ms_pers = 0.0f;
      b->persistent = 0;
      rc = trial(ms_graph);
      if (!rc) {
        b->persistent = 1;
        rc = trial(ms_pers);
      }
      b->persistent = (!rc && ms_pers < ms_graph) ? 1 : 0;
    }
  }
  batch_invalidate_graph(b);
  if (rc) return rc;
  if (chosen) {
    chosen[0] = b->wpb;
    chosen[1] = b->cached_div;
    for (int m = 2; m <= 4; ++m) chosen[m] = b->class_mode[m];
    chosen[5] = b->persistent;
  }
  return ok();
}

// As profile_steps, over all runs of a batch.
static int batch_profile_steps(ibm_batch *b, int64_t n, double *ms_per_phase, double *kernel_ms) {
  if (n < 1 || n > 4096) return fail(IBM_ERR_INVALID_ARG, "profile 1..4096 steps");
  int rc = batch_sync_tables(b);
  if (rc) return rc;
  ibm_lattice *r0 = b->runs[0];
  EventPool pool;
  std::vector<hipEvent_t> ev((size_t)n * 4);
  std::vector<ibm::DispatchTimer> kt(kernel_ms ? (size_t)n : 0);
  for (auto &e : ev) IBM_HIP(pool.make(&e));
  for (auto &t : kt) {
    IBM_HIP(pool.make(&t.start));
    IBM_HIP(pool.make(&t.stop));
  }
  hipStream_t s = b->stream;
  for (int64_t k = 0; k < n; ++k) {
    for (ibm_lattice *lat : b->runs)
      if (lat->has_mem && lat->since_recenter >= lat->recenter_every) {
        ibm::launch_recenter(lat->M, s);
        lat->since_recenter = 0;
        if (lat->overlap) lat->slab_stale = true;
      }
    hipEvent_t *e = &ev[(size_t)k * 4];
    const int src = (int)(r0->steps & 1), par = src;
    const int advect = (r0->ab2 && batch_prev_u(b)) ? 1 : 0;
    IBM_HIP(hipEventRecord(e[0], s));
    ibm::launch_batch_spread(b->B, par, s);
    IBM_HIP(hipEventRecord(e[1], s));
    ibm::launch_batch_collide_stream(b->B, r0->storage, src, par, r0->eq_linear != 0, s,
                                     kernel_ms ? &kt[(size_t)k] : nullptr);
    IBM_HIP(hipEventRecord(e[2], s));
    ibm::launch_batch_interp(b->B, r0->storage, src ^ 1, par, advect, s);
    IBM_HIP(hipEventRecord(e[3], s));
    for (ibm_lattice *lat : b->runs) {
      lat->steps += 1;
      lat->since_recenter += 1;
      if (lat->ab2 && lat->has_mem) lat->have_prev_u = true;
    }
  }
  IBM_HIP(hipGetLastError());
  IBM_HIP(hipStreamSynchronize(s));
  double acc[IBM_N_PHASES] = {0.0, 0.0, 0.0, 0.0}, kacc = 0.0;
  const int phase_of[3] = {IBM_PHASE_SPREAD, IBM_PHASE_LBM, IBM_PHASE_INTERP};
  for (int64_t k = 0; k < n; ++k) {
    hipEvent_t *e = &ev[(size_t)k * 4];
    for (int p = 0; p < 3; ++p) {
      float ms = 0.0f;
      IBM_HIP(hipEventElapsedTime(&ms, e[p], e[p + 1]));
      acc[phase_of[p]] += ms;
    }
    if (kernel_ms) {
      float ms = 0.0f;
      IBM_HIP(hipEventElapsedTime(&ms, kt[(size_t)k].start, kt[(size_t)k].stop));
      kacc += ms;
    }
  }
  if (ms_per_phase)
    for (int p = 0; p < IBM_N_PHASES; ++p) ms_per_phase[p] = acc[p] / (double)n;
  if (kernel_ms) *kernel_ms = kacc / (double)n;
  return ok();
}

int ibm_batch_profile_step(ibm_batch *b, int64_t n, double *ms_per_phase) {
  if (!b || !ms_per_phase) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  return batch_profile_steps(b, n, ms_per_phase, nullptr);
}

int ibm_batch_profile_lattice_kernel(ibm_batch *b, int64_t n, double *ms) {
  if (!b || !ms) return fail(IBM_ERR_INVALID_ARG, "NULL argument");
  return batch_profile_steps(b, n, nullptr, ms);
}

int ibm_batch_destroy(ibm_batch *b) {
  if (!b) return ok();
  (void)hipStreamSynchronize(b->stream);
  batch_invalidate_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
  return ok();
}

}  // extern "C"
