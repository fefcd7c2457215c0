// Tuned CPU kernel of libdisthist: the same histograms on the host's cores,
// for comparison with the GPU path and for hosts without a GPU. Following the
// CPU design of the paper (Sec. 3.1): the pairs are cut into cache-sized
// tiles (triangular tiles on the diagonal of an intra-species histogram),
// coordinates are kept per tile as separate x, y, z arrays so that the
// compiler vectorizes the distance loop without intrinsics, the bin indices of
// one row of a tile go to a small buffer first and are then scattered into a
// thread-private histogram. Threads take tiles from a shared counter.
//
// Arithmetic: the canonical sequence of the library (see disthist.h) in the
// working precision; binary64 results are therefore identical to the GPU
// path's. binary32 rounds the coordinates and the binary64 constants once.
#include "disthist.h"
#include "dh_internal.h"

#include <sched.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

namespace {

template <typename T>
struct CpuGeo {
  T s, nb;
  T L[3], iL[3];
  T ax, bx, by, cx, cy, cz, h11, h12, h13, h22, h23, h33;
  T sh[dh::kShifts][3];
};

template <typename T>
CpuGeo<T> make_geo(const dh::FrameParams &f) {
  CpuGeo<T> g;
  g.s = static_cast<T>(f.s);
  g.nb = static_cast<T>(f.n_bins);
  for (int c = 0; c < 3; ++c) {
    g.L[c] = static_cast<T>(f.L[c]);
    g.iL[c] = static_cast<T>(f.iL[c]);
  }
  g.ax = static_cast<T>(f.ax); g.bx = static_cast<T>(f.bx); g.by = static_cast<T>(f.by);
  g.cx = static_cast<T>(f.cx); g.cy = static_cast<T>(f.cy); g.cz = static_cast<T>(f.cz);
  g.h11 = static_cast<T>(f.h11); g.h12 = static_cast<T>(f.h12); g.h13 = static_cast<T>(f.h13);
  g.h22 = static_cast<T>(f.h22); g.h23 = static_cast<T>(f.h23); g.h33 = static_cast<T>(f.h33);
  for (int m = 0; m < dh::kShifts; ++m)
    for (int c = 0; c < 3; ++c) g.sh[m][c] = static_cast<T>(f.shift64[m][c]);
  return g;
}

// Bin index (n_bins for out of range) of particle (xi, yi, zi) against
// particles [0, n) of the j arrays; the loop is written for the vectorizer.
template <typename T, int BOX>
void row(T xi, T yi, T zi, const T *__restrict__ xj, const T *__restrict__ yj,
         const T *__restrict__ zj, int n, const CpuGeo<T> &g, int32_t n_bins,
         int32_t *__restrict__ idx) {
  const T s = g.s, nb = g.nb;
  const T L0 = g.L[0], L1 = g.L[1], L2 = g.L[2], iL0 = g.iL[0], iL1 = g.iL[1], iL2 = g.iL[2];
  const T ax = g.ax, bx = g.bx, by = g.by, cx = g.cx, cy = g.cy, cz = g.cz;
  const T h11 = g.h11, h12 = g.h12, h13 = g.h13, h22 = g.h22, h23 = g.h23, h33 = g.h33;
#pragma clang loop vectorize(enable)
  for (int j = 0; j < n; ++j) {
    T dx = xj[j] - xi, dy = yj[j] - yi, dz = zj[j] - zi;
    if constexpr (BOX == dh::kBoxOrtho) {
      const T n0 = std::rint(dx * iL0), n1 = std::rint(dy * iL1), n2 = std::rint(dz * iL2);
      dx = std::fma(-L0, n0, dx);
      dy = std::fma(-L1, n1, dy);
      dz = std::fma(-L2, n2, dz);
    } else if constexpr (BOX == dh::kBoxTric || BOX == dh::kBoxTricSearch) {
      const T sc = dz * h33;
      const T sb = std::fma(dz, h23, dy * h22);
      const T sa = std::fma(dz, h13, std::fma(dy, h12, dx * h11));
      const T na = std::rint(sa), nbb = std::rint(sb), nc = std::rint(sc);
      dz = std::fma(-cz, nc, dz);
      dy = std::fma(-cy, nc, std::fma(-by, nbb, dy));
      dx = std::fma(-cx, nc, std::fma(-bx, nbb, std::fma(-ax, na, dx)));
    }
    T q = std::fma(dz, dz, std::fma(dy, dy, dx * dx));
    if constexpr (BOX == dh::kBoxTricSearch) {
#pragma clang loop unroll(full)
      for (int m = 0; m < dh::kShifts; ++m) {
        const T vx = dx + g.sh[m][0], vy = dy + g.sh[m][1], vz = dz + g.sh[m][2];
        const T v = std::fma(vz, vz, std::fma(vy, vy, vx * vx));
        q = v < q ? v : q;
      }
    }
    const T t = std::sqrt(q) * s;
    idx[j] = t < nb ? static_cast<int32_t>(t) : n_bins;
  }
}

struct Tile {
  int32_t hist;
  int64_t i0, i1, j0, j1;
  bool diag;
};

template <typename T, int BOX>
void run(const std::vector<T> &X, const std::vector<T> &Y, const std::vector<T> &Z,
         const std::vector<Tile> &tiles, const CpuGeo<T> &g, int32_t n_hist, int32_t n_bins,
         int n_threads, uint64_t *out) {
  const size_t stride = static_cast<size_t>(n_bins) + 1;  // + the out-of-range slot
  std::vector<std::vector<uint64_t>> priv(n_threads);
  std::atomic<size_t> next{0};
  auto worker = [&](int w) {
    std::vector<uint64_t> &h = priv[w];
    h.assign(static_cast<size_t>(n_hist) * stride, 0);
    std::vector<int32_t> idx;
    for (;;) {
      const size_t k = next.fetch_add(1, std::memory_order_relaxed);
      if (k >= tiles.size()) break;
      const Tile &tl = tiles[k];
      uint64_t *hh = h.data() + static_cast<size_t>(tl.hist) * stride;
      idx.resize(static_cast<size_t>(tl.j1 - tl.j0));
      for (int64_t i = tl.i0; i < tl.i1; ++i) {
        const int64_t j0 = tl.diag ? i + 1 : tl.j0;
        const int n = static_cast<int>(tl.j1 - j0);
        if (n <= 0) continue;
        row<T, BOX>(X[i], Y[i], Z[i], X.data() + j0, Y.data() + j0, Z.data() + j0, n, g, n_bins,
                    idx.data());
        for (int j = 0; j < n; ++j) ++hh[idx[j]];
      }
    }
  };
  std::vector<std::thread> pool;
  for (int w = 1; w < n_threads; ++w) pool.emplace_back(worker, w);
  worker(0);
  for (auto &th : pool) th.join();
  for (int32_t hh = 0; hh < n_hist; ++hh)
    for (int32_t b = 0; b < n_bins; ++b) {
      uint64_t v = 0;
      for (int w = 0; w < n_threads; ++w) v += priv[w][static_cast<size_t>(hh) * stride + b];
      out[static_cast<size_t>(hh) * n_bins + b] = v;
    }
}

// Tile edge: coordinates of a j-tile (3 arrays), its index buffer and one
// thread-private histogram should stay in a core's L2 (Sec. 3.1, Eq. 6
// sizes the tile from the L2 size the same way); 1 MiB L2 assumed.
int64_t tile_edge(int32_t n_bins, size_t coord_bytes, int32_t n_hist) {
  const int64_t l2 = 1 << 20, reserve = 16 << 10;
  const int64_t hist = 8 * (static_cast<int64_t>(n_bins) + 1) * std::min(n_hist, 3);
  const int64_t room = std::max<int64_t>(l2 - reserve - hist, 64 << 10);
  const int64_t per = 3 * static_cast<int64_t>(coord_bytes) + 4;
  return std::max<int64_t>(256, std::min<int64_t>(8192, room / per / 256 * 256));
}

// The CPUs this process may run on (its affinity mask), at most
// OMP_NUM_THREADS when that is set (the usual share of a node).
int32_t default_threads() {
  int32_t n = 0;
  cpu_set_t set;
  if (sched_getaffinity(0, sizeof set, &set) == 0) n = CPU_COUNT(&set);
  if (n <= 0) n = static_cast<int32_t>(std::max(1u, std::thread::hardware_concurrency()));
  if (const char *e = std::getenv("OMP_NUM_THREADS")) {
    const long v = std::strtol(e, nullptr, 10);
    if (v > 0 && v < n) n = static_cast<int32_t>(v);
  }
  return n;
}

}  // namespace

extern "C" int dh_cpu_histo(const double *coords, const int64_t *offsets, int32_t n_species,
                            int32_t box_type, const double *box, double r_max, int32_t n_bins,
                            int32_t precision, int32_t n_threads, uint64_t *out,
                            uint64_t *out_of_range) {
  const int rc = dh_check_args(coords, offsets, n_species, box_type, box, r_max, n_bins, precision);
  if (rc) return rc;
  const int64_t n = offsets[n_species];
  if (!out || (n > 0 && !coords) || n_threads < 0) return DH_EINVAL;
  if (n_threads == 0) n_threads = default_threads();
  n_threads = std::min(n_threads, 1024);
  dh::FrameParams fp;
  const int kind = dh::frame_constants(box_type, box, r_max, n_bins, fp);
  const int32_t n_hist = n_species * (n_species + 1) / 2;

  // tiles: intra-species triangles first, then cross pairs (library order)
  const size_t cb = precision == DH_FP64 ? 8 : 4;
  const int64_t B = tile_edge(n_bins, cb, n_hist);
  std::vector<Tile> tiles;
  std::vector<uint64_t> pairs(n_hist, 0);
  int32_t h = 0;
  for (int32_t sp = 0; sp < n_species; ++sp, ++h) {
    const int64_t a = offsets[sp], e = offsets[sp + 1];
    pairs[h] = static_cast<uint64_t>(e - a) * static_cast<uint64_t>(e - a > 0 ? e - a - 1 : 0) / 2;
    for (int64_t i0 = a; i0 < e; i0 += B)
      for (int64_t j0 = i0; j0 < e; j0 += B)
        tiles.push_back({h, i0, std::min(i0 + B, e), j0, std::min(j0 + B, e), j0 == i0});
  }
  for (int32_t sp = 0; sp < n_species; ++sp)
    for (int32_t tp = sp + 1; tp < n_species; ++tp, ++h) {
      pairs[h] = static_cast<uint64_t>(offsets[sp + 1] - offsets[sp]) *
                 static_cast<uint64_t>(offsets[tp + 1] - offsets[tp]);
      for (int64_t i0 = offsets[sp]; i0 < offsets[sp + 1]; i0 += B)
        for (int64_t j0 = offsets[tp]; j0 < offsets[tp + 1]; j0 += B)
          tiles.push_back({h, i0, std::min(i0 + B, offsets[sp + 1]), j0,
                           std::min(j0 + B, offsets[tp + 1]), false});
    }
  // large tiles first, then the rest (balance at the end)
  std::stable_sort(tiles.begin(), tiles.end(), [](const Tile &x, const Tile &y) {
    return (x.i1 - x.i0) * (x.j1 - x.j0) > (y.i1 - y.i0) * (y.j1 - y.j0);
  });
  n_threads = static_cast<int32_t>(std::min<size_t>(n_threads, std::max<size_t>(1, tiles.size())));

  auto go = [&](auto zero) {
    using T = decltype(zero);
    std::vector<T> X(n), Y(n), Z(n);
    for (int64_t i = 0; i < n; ++i) {
      X[i] = static_cast<T>(coords[3 * i]);
      Y[i] = static_cast<T>(coords[3 * i + 1]);
      Z[i] = static_cast<T>(coords[3 * i + 2]);
    }
    const CpuGeo<T> g = make_geo<T>(fp);
    switch (kind) {
      case dh::kBoxNone: run<T, dh::kBoxNone>(X, Y, Z, tiles, g, n_hist, n_bins, n_threads, out); break;
      case dh::kBoxOrtho: run<T, dh::kBoxOrtho>(X, Y, Z, tiles, g, n_hist, n_bins, n_threads, out); break;
      case dh::kBoxTric: run<T, dh::kBoxTric>(X, Y, Z, tiles, g, n_hist, n_bins, n_threads, out); break;
      default: run<T, dh::kBoxTricSearch>(X, Y, Z, tiles, g, n_hist, n_bins, n_threads, out); break;
    }
  };
  if (precision == DH_FP64)
    go(0.0);
  else
    go(0.0f);
  if (out_of_range)
    for (int32_t hh = 0; hh < n_hist; ++hh) {
      uint64_t in = 0;
      for (int32_t b = 0; b < n_bins; ++b) in += out[static_cast<size_t>(hh) * n_bins + b];
      out_of_range[hh] = pairs[hh] - in;
    }
  return DH_OK;
}
