// CPU check of the population addressing of the collide-stream row form:
// for each lattice shape given on the command line (nx ny nz), the offsets
// the row form forms with 32-bit group-row indices (grow32, rowoff and the
// per-direction table pst) must equal the 64-bit offsets of the reference
// formula pidx and lie inside one population buffer, for every population
// and every 4-node segment of the rows checked: all rows when there are at
// most 2^20 of them, else the first and last 4096 rows, the rows around
// every 2^k boundary and a strided sample.  Runs on the host only (the
// addressing functions are host-callable).  Prints one line per shape;
// exit status 1 on any mismatch.
#include <cstdio>
#include <cstdlib>
#include <set>
#include <vector>

#include "common.h"
#include "lbm_device.h"

using namespace ibm;

static int check_shape(int nx, int ny, int nz) {
  const PopGeometry pg = pop_geometry(nx, ny, nz);
  LatDev L{};
  L.nx = nx;
  L.ny = ny;
  L.nz = nz;
  L.nxs = pg.nxs;
  L.gsh = pg.gsh;
  L.tpr = pg.tpr;
  L.rpw = pg.rpw;
  for (int i = 0; i < Q; ++i) L.pst[i] = (long long)i * ((long long)L.nxs << L.gsh);
  const long long rows = (long long)ny * nz;
  std::printf("%d x %d x %d: nxs %d, %d rows per group, row form %s", nx, ny, nz, pg.nxs,
              1 << pg.gsh, pg.tpr ? "yes" : "no");
  if (!pg.tpr) {
    // the row form is off exactly where its 32-bit group-row index could
    // overflow or a row does not fit one wavefront
    const long long g = 1LL << pg.gsh;
    const bool fits = pg.nxs / 4 <= 64 && (rows + g - 1) / g * g * Q < (1LL << 32);
    std::printf(fits ? "  MISMATCH: row form off although it fits\n" : "\n");
    return fits ? 1 : 0;
  }
  std::vector<long long> sample;
  if (rows <= (1LL << 20)) {
    for (long long r = 0; r < rows; ++r) sample.push_back(r);
  } else {
    std::set<long long> s;
    for (long long r = 0; r < 4096; ++r) {
      s.insert(r);
      s.insert(rows - 1 - r);
    }
    for (int k = 10; k < 40; ++k)
      for (long long d = -3; d <= 3; ++d) {
        const long long r = (1LL << k) + d;
        if (r >= 0 && r < rows) s.insert(r);
      }
    for (long long r = 0; r < rows; r += 997) s.insert(r);
    sample.assign(s.begin(), s.end());
  }
  long long bad = 0, checked = 0, maxoff = 0;
  for (long long r : sample)
    for (int x = 0; x < pg.nxs; x += 4)
      for (int i = 0; i < Q; ++i) {
        const long long ref = pidx(L, i, r, x);
        const long long got = L.pst[i] + (long long)rowoff(L, (unsigned)r, x);
        ++checked;
        if (got != ref || got < 0 || got + 3 >= pg.pop_elems) {
          if (bad < 5)
            std::printf("\n  row %lld x %d i %d: row form %lld, reference %lld, buffer %lld", r, x, i,
                        got, ref, pg.pop_elems);
          ++bad;
        }
        if (got > maxoff) maxoff = got;
      }
  std::printf(", %lld offsets checked, largest %lld of %lld: %s\n", checked, maxoff + 3,
              pg.pop_elems, bad ? "MISMATCH" : "ok");
  return bad ? 1 : 0;
}

int main(int argc, char **argv) {
  int fails = 0;
  for (int a = 1; a + 2 < argc; a += 3)
    fails += check_shape(std::atoi(argv[a]), std::atoi(argv[a + 1]), std::atoi(argv[a + 2]));
  return fails ? 1 : 0;
}
