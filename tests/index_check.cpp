// Host check of the sweeps' index arithmetic (fv_index.hpp) against its plain
// definition: divisions of the flattened position.  Prints "ok" or the first
// mismatch and exits non-zero.
#include <cstdio>
#include <initializer_list>

#include "fv_index.hpp"

using namespace rfv;

static int check_x(int nx, int ny, int nz, int nt) {
  const int lx = nx + 4, total = lx * ny * nz, c = nt - 4;
  const int tiles = (total + c - 1) / c;
  for (int lt = 0; lt < tiles; ++lt) {
    for (int tid = 0; tid < nt; ++tid) {
      const int f = lt * c - 2 + tid;
      const bool valid = f >= 0 && f < total;
      const int fc = f < 0 ? 0 : (f >= total ? total - 1 : f);
      const int row = fc / lx, il = fc % lx, j = row % ny, k = row / ny;
      const XPos p = x_position(tid, lt * c - 2, lx, ny, nz);
      const int f0 = lt * c - 2 < 0 ? 0 : lt * c - 2;
      const bool ok = p.valid == valid && p.il == il && p.j0 + p.dj == j && p.k0 + p.dk == k &&
                      p.j0 == (f0 / lx) % ny && p.k0 == (f0 / lx) / ny;
      if (!ok) {
        std::printf("x_position mismatch n=(%d,%d,%d) nt=%d tile=%d tid=%d: got il=%d j=%d k=%d "
                    "valid=%d, want il=%d j=%d k=%d valid=%d\n", nx, ny, nz, nt, lt, tid, p.il,
                    p.j0 + p.dj, p.k0 + p.dk, (int)p.valid, il, j, k, (int)valid);
        return 1;
      }
    }
  }
  return 0;
}

static int check_face() {
  for (int n = 1; n <= 9; ++n)
    for (int j = -2; j < n + 2; ++j) {
      const int t = face_index(j, n, FACE_TRANSMISSIVE, FACE_TRANSMISSIVE);
      const int p = face_index(j, n, FACE_PERIODIC, FACE_PERIODIC);
      const int h = face_index(j, n, FACE_HALO, FACE_HALO);
      const int want_t = j < 0 ? 0 : (j >= n ? n - 1 : j);
      const int want_p = ((j % n) + n) % n;
      if (t != want_t || h != j || (n >= 2 && p != want_p)) {
        std::printf("face_index mismatch n=%d j=%d\n", n, j);
        return 1;
      }
    }
  return 0;
}

int main() {
  if (check_face()) return 1;
  const int nxs[] = {1, 2, 3, 5, 17, 32, 61, 124, 125, 252, 253, 256, 300, 512};
  const int nys[] = {1, 3, 7, 16};
  const int nzs[] = {1, 2, 5};
  for (int nt : {128, 256})
    for (int nx : nxs)
      for (int ny : nys)
        for (int nz : nzs)
          if (check_x(nx, ny, nz, nt)) return 1;
  std::printf("ok\n");
  return 0;
}
