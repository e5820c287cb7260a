// Host check of the CG update tiles (test infrastructure): for every order
// and candidate tile shape, the element-column positions of all threads of
// all tiles on a small box own every element-local node exactly once (live,
// below their plane range's end), and every LDS slot a thread reads for an
// x copy inside its tile is a slot that the x neighbour's thread writes.
// For the linear tile (every order that has one, on boxes of one element
// across in x, y or z too): each item's boundary flag, multiplicity and set
// of copy addresses equal those found directly from the node's element and
// position, and every node is an item of exactly one thread.
// Compiled for the host with hipcc by tests/test_update_tiles_host.py.
#include <algorithm>
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

// The copies of node (e, i, j, k) found directly: along each direction the
// node itself, or both sides of a face shared with the neighbour element.
template <int N1>
int check_linear_box(int nx, int ny, int nz) {
  constexpr int N = N1 - 1;
  constexpr int64_t NP = (int64_t)N1 * N1 * N1;
  const Box b = Box::make(nx, ny, nz, N);
  const int64_t L = b.L();
  const int64_t tiles = vec_grid_blocks(L);
  std::vector<int> seen(L, 0);
  int bad = 0;
  for (int64_t t = 0; t < tiles; ++t)
    for (int tid = 0; tid < kVecThreads; ++tid) {
      const LinItems<N1> P(b, t, tid);
      for (int u = 0; u < kVecItems; ++u) {
        const typename LinItems<N1>::Item it = P.item(u);
        const int64_t raw = t * kVecTile + tid + (int64_t)u * kVecThreads;
        if ((int64_t)it.raw != raw || it.live != (raw < L)) { ++bad; continue; }
        if (!it.live) {
          if ((int64_t)it.idx != L - 1 || it.sh != 0 || it.lo != it.idx || it.upd) ++bad;
          continue;
        }
        ++seen[raw];
        const int64_t e = raw / NP, loc = raw % NP;
        const int i = (int)(loc % N1), j = (int)(loc / N1 % N1), k = (int)(loc / (N1 * N1));
        const int ex = (int)(e % nx), ey = (int)(e / nx % ny), ez = (int)(e / ((int64_t)nx * ny));
        const bool boundary = (i == 0 && ex == 0) || (i == N && ex == nx - 1) || (j == 0 && ey == 0) ||
                              (j == N && ey == ny - 1) || (k == 0 && ez == 0) || (k == N && ez == nz - 1);
        // per direction: (element coordinate, local index) of each copy
        int cx[2][2], cy[2][2], cz[2][2], mx = 1, my = 1, mz = 1;
        cx[0][0] = ex; cx[0][1] = i; cy[0][0] = ey; cy[0][1] = j; cz[0][0] = ez; cz[0][1] = k;
        if (i == 0 && ex > 0) { mx = 2; cx[1][0] = ex - 1; cx[1][1] = N; }
        if (i == N && ex < nx - 1) { mx = 2; cx[1][0] = ex + 1; cx[1][1] = 0; }
        if (j == 0 && ey > 0) { my = 2; cy[1][0] = ey - 1; cy[1][1] = N; }
        if (j == N && ey < ny - 1) { my = 2; cy[1][0] = ey + 1; cy[1][1] = 0; }
        if (k == 0 && ez > 0) { mz = 2; cz[1][0] = ez - 1; cz[1][1] = N; }
        if (k == N && ez < nz - 1) { mz = 2; cz[1][0] = ez + 1; cz[1][1] = 0; }
        std::vector<int64_t> want;
        for (int a = 0; a < mx; ++a)
          for (int c = 0; c < my; ++c)
            for (int d = 0; d < mz; ++d) {
              const int64_t ee = ((int64_t)cz[d][0] * ny + cy[c][0]) * nx + cx[a][0];
              want.push_back(ee * NP + ((int64_t)cz[d][1] * N1 + cy[c][1]) * N1 + cx[a][1]);
            }
        std::sort(want.begin(), want.end());
        std::vector<int64_t> got;
        for (int q = 0; q < 8; ++q)
          if (LinItems<N1>::has_copy(it.sh, q)) got.push_back((int64_t)(uint32_t)(it.lo + P.off(q)));
        const bool ascending = std::is_sorted(got.begin(), got.end());
        if (it.upd == boundary || (1 << __builtin_popcount(it.sh)) != mx * my * mz || got != want ||
            !ascending || (int64_t)it.idx != raw)
          ++bad;
      }
    }
  for (int64_t a = 0; a < L; ++a)
    if (seen[a] != 1) ++bad;
  if (bad) std::printf("linear tile, order %d, box %dx%dx%d: %d violations\n", N, nx, ny, nz, bad);
  return bad;
}

template <int N1>
int check_linear() {
  return check_linear_box<N1>(3, 2, 2) + check_linear_box<N1>(1, 3, 2) + check_linear_box<N1>(2, 1, 3) +
         check_linear_box<N1>(2, 3, 1) + check_linear_box<N1>(1, 1, 1);
}

int main() {
  static_assert(kUpdVariants == 4, "four candidate shapes");
  const int bad = check_order<2>() + check_order<3>() + check_order<4>() + check_order<5>() +
                  check_order<6>() + check_order<7>() + check_order<8>() + check_order<9>() +
                  check_order<10>() + check_order<11>() + check_order<12>() + check_order<13>() +
                  check_linear<10>() + check_linear<11>() + check_linear<12>() + check_linear<13>() +
                  check_linear<14>() + check_linear<15>() + check_linear<16>();
  std::printf("%s\n", bad ? "FAIL" : "OK");
  return bad ? 1 : 0;
}
