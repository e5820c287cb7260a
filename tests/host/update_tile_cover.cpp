// Host check of the CG update tiles (test infrastructure): for every order
// and candidate tile shape, the element-column positions of all threads of
// all tiles on a small box own every element-local node exactly once (live,
// below their plane range's end), and every LDS slot a thread reads for an
// x copy inside its tile is a slot that the x neighbour's thread writes.
// Compiled for the host with hipcc by tests/test_update_tiles_host.py.
#include <cstdio>
#include <vector>

#include "sem_cg_dev.h"

using namespace semk;

template <int N1, typename TV, int V>
int check(int nx, int ny, int nz) {
  using U = UpdTile<N1, TV, V>;
  if constexpr (U::LINEAR) {
    return 0;
  } else {
    const Box b = Box::make(nx, ny, nz, N1 - 1);
    const int64_t L = b.L();
    std::vector<int> owned(L, 0);
    const int64_t tiles = upd_num_tiles(b, sizeof(TV) == 8, V);
    int bad = 0;
    for (int64_t t = 0; t < tiles; ++t) {
      std::vector<int> written(U::LDS > 1 ? U::LDS : 1, 0);
      for (int tid = 0; tid < U::BLOCK; ++tid) {
        const ColumnPos<N1, TV, V> p(b, t, tid);
        if (tid < U::THREADS && U::EPT > 1)
          for (int kk = 0; kk < U::KN; ++kk) written[((p.el * U::KS + p.ks) * U::KN + kk) * U::COLS + p.col] = 1;
        for (int kk = 0; kk < U::KN; ++kk) {
          const int k = p.kb + kk;
          if (p.live && k < p.kend) {
            const int64_t a = p.col0 + (int64_t)k * U::COLS;
            if (a < 0 || a >= L) ++bad;
            else ++owned[a];
          }
        }
      }
      for (int tid = 0; tid < U::THREADS; ++tid) {
        const ColumnPos<N1, TV, V> p(b, t, tid);
        if (!p.x_in) continue;
        const int xo = ((p.i == 0 ? p.el - 1 : p.el + 1) * U::KS + p.ks) * U::KN * U::COLS + p.j * N1 +
                       (U::N - p.i);
        for (int kk = 0; kk < U::KN; ++kk) {
          const int s = xo + kk * U::COLS;
          if (s < 0 || s >= U::LDS || !written[s]) ++bad;
        }
      }
    }
    for (int64_t a = 0; a < L; ++a)
      if (owned[a] != 1) ++bad;
    if (bad) std::printf("order %d %s shape %d: %d violations\n", N1 - 1, sizeof(TV) == 8 ? "f64" : "f32", V, bad);
    return bad;
  }
}

template <int N1, typename TV>
int check_all(int nx, int ny, int nz) {
  return check<N1, TV, 0>(nx, ny, nz) + check<N1, TV, 1>(nx, ny, nz) + check<N1, TV, 2>(nx, ny, nz) +
         check<N1, TV, 3>(nx, ny, nz);
}

template <int N1>
int check_order() {
  // a ragged box: several tiles of every shape, the last one partly empty
  const int n = N1 <= 4 ? 6 : (N1 <= 9 ? 4 : 3);
  return check_all<N1, double>(n + 1, n, n - 1) + check_all<N1, float>(n + 1, n, n - 1);
}

int main() {
  static_assert(kUpdVariants == 4, "four candidate shapes");
  const int bad = check_order<2>() + check_order<3>() + check_order<4>() + check_order<5>() +
                  check_order<6>() + check_order<7>() + check_order<8>() + check_order<9>() +
                  check_order<10>() + check_order<11>() + check_order<12>() + check_order<13>();
  std::printf("%s\n", bad ? "FAIL" : "OK");
  return bad ? 1 : 0;
}
