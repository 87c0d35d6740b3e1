// Spherical capsule meshes by icosahedron subdivision (Sec. II.D, Fig. 3):
// halve every edge, push the new node radially onto the sphere, split each
// face into four; repeat.
#include <cmath>
#include <cstdint>
#include <map>
#include <utility>
#include <vector>

#include "ibm_lbm.h"

extern "C" int ibm_icosphere_size(int level, int *nn, int *nf) {
  if (!nn || !nf || level < 0 || level > 7) return IBM_ERR_INVALID_ARG;
  long long f = 20;
  for (int l = 0; l < level; ++l) f *= 4;
  *nf = (int)f;
  *nn = (int)(f / 2 + 2);  // Euler: 2 N_n = N_f + 4
  return IBM_OK;
}

extern "C" int ibm_icosphere(int level, double r, double cx, double cy, double cz, double *xyz,
                             int32_t *tri) {
  int nn = 0, nf = 0;
  if (ibm_icosphere_size(level, &nn, &nf) != IBM_OK || !xyz || !tri || !(r > 0.0))
    return IBM_ERR_INVALID_ARG;
  const double t = 0.5 * (1.0 + std::sqrt(5.0));
  std::vector<double> v = {-1, t, 0, 1, t, 0, -1, -t, 0, 1, -t, 0,
                           0, -1, t, 0, 1, t, 0, -1, -t, 0, 1, -t,
                           t, 0, -1, t, 0, 1, -t, 0, -1, -t, 0, 1};
  // the 20 faces of this vertex numbering, counter-clockwise from outside
  std::vector<int> f = {0, 11, 5, 0, 5, 1, 0, 1, 7, 0, 7, 10, 0, 10, 11,
                        1, 5, 9, 5, 11, 4, 11, 10, 2, 10, 7, 6, 7, 1, 8,
                        3, 9, 4, 3, 4, 2, 3, 2, 6, 3, 6, 8, 3, 8, 9,
                        4, 9, 5, 2, 4, 11, 6, 2, 10, 8, 6, 7, 9, 8, 1};
  auto unit = [&](int k) {
    double *p = &v[3 * (size_t)k];
    const double s = 1.0 / std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    p[0] *= s;
    p[1] *= s;
    p[2] *= s;
  };
  for (int k = 0; k < 12; ++k) unit(k);
  for (int l = 0; l < level; ++l) {
    std::map<std::pair<int, int>, int> mid;
    auto midpoint = [&](int a, int b) {
      const std::pair<int, int> key(std::min(a, b), std::max(a, b));
      auto it = mid.find(key);
      if (it != mid.end()) return it->second;
      const int id = (int)(v.size() / 3);
      for (int d = 0; d < 3; ++d) v.push_back(0.5 * (v[3 * (size_t)a + d] + v[3 * (size_t)b + d]));
      unit(id);
      mid.emplace(key, id);
      return id;
    };
    std::vector<int> g;
    g.reserve(f.size() * 4);
    for (size_t j = 0; j < f.size(); j += 3) {
      const int a = f[j], b = f[j + 1], c = f[j + 2];
      const int ab = midpoint(a, b), bc = midpoint(b, c), ca = midpoint(c, a);
      const int quad[12] = {a, ab, ca, b, bc, ab, c, ca, bc, ab, bc, ca};
      g.insert(g.end(), quad, quad + 12);
    }
    f.swap(g);
  }
  if ((int)(v.size() / 3) != nn || (int)(f.size() / 3) != nf) return IBM_ERR_INVALID_ARG;
  for (int k = 0; k < nn; ++k) {
    xyz[3 * k + 0] = cx + r * v[3 * (size_t)k + 0];
    xyz[3 * k + 1] = cy + r * v[3 * (size_t)k + 1];
    xyz[3 * k + 2] = cz + r * v[3 * (size_t)k + 2];
  }
  for (int j = 0; j < nf * 3; ++j) tri[j] = f[j];
  return IBM_OK;
}
