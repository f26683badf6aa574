// Driver of the library's host-only arithmetic (csrc/host.cpp) for the
// sanitizer test: built with the host compiler and AddressSanitizer /
// UndefinedBehaviorSanitizer, it checks the work-plan and geometry rules
// itself and evaluates the tridiagonal eigenproblems and SLQ quadratures the
// Python side reads back.  Commands on stdin, one per line:
//   plans                       check every sweep plan on a grid of sizes
//   wide                        check the wide sweep's tiled schedule
//   geometry                    check the operand geometry of every precision
//   tridiag m d_0..d_{m-1} e_0..e_{m-2}
//                               eigenvalues and first eigenvector row
//   slq m znorm2 a_0..a_{m-1} b_0..b_{m-2}
//                               status and quadrature value
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <iostream>
#include <string>
#include <vector>

#include "../../paper_1706_00241_amd/csrc/host.h"

using namespace dcg;

#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      std::abort();                                                       \
    }                                                                     \
  } while (0)

// Every block offset 0..nb/2 lies in exactly one chunk, the grid is one work
// item per (row block, chunk), and the partial buffers sized for the largest
// item target hold those of every smaller one.
static void check_plan(const MatvecPlan &p, int64_t n_pad, int blk) {
  CHECK(p.blk == blk && int64_t(p.nb) * blk == n_pad);
  CHECK(p.dmax == p.nb / 2 && p.chunk >= 1 && p.nchunk >= 1);
  CHECK(int64_t(p.nchunk) * p.chunk >= p.dmax + 1);
  CHECK(int64_t(p.nchunk - 1) * p.chunk < p.dmax + 1);
  CHECK(p.grid == int64_t(p.nb) * p.nchunk);
}

static long plans() {
  long count = 0;
  for (int64_t n_pad = 256; n_pad <= (int64_t(1) << 22); n_pad = n_pad * 3 / 2 / 256 * 256 + 256) {
    for (int blk : {128, 256}) {
      if (n_pad % blk) continue;
      const MatvecPlan pmax = make_plan(n_pad, blk, kSweepItemsMax);
      for (int items = kSweepItemsMin; items <= kSweepItemsMax; items *= 2) {
        const MatvecPlan p = make_plan(n_pad, blk, items);
        check_plan(p, n_pad, blk);
        CHECK(p.nchunk <= pmax.nchunk);
        for (int mv : {1, 4})
          CHECK(size_t(2 * p.nchunk + p.dmax) * size_t(n_pad) * mv <=
                matvec_partial_floats(n_pad, mv, blk));
        ++count;
      }
    }
    if (n_pad % 128 == 0) {
      const MatvecPlan emax = exact_plan(n_pad, kSweepItemsMax);
      for (int items = kSweepItemsMin; items <= kSweepItemsMax; items *= 2) {
        const MatvecPlan p = exact_plan(n_pad, items);
        check_plan(p, n_pad, 128);
        CHECK(p.nchunk <= emax.nchunk);
        CHECK(size_t(p.nchunk + p.dmax) * size_t(n_pad) <= exact_partial_doubles(n_pad));
        ++count;
      }
    }
  }
  return count;
}

// The augmented operands fit their stored width: bf16 / fp16 points take
// d + 6 entries (the point, three norm terms on each side), split bf16 4d + 6,
// FP32 as three bf16 terms 6d + 6, FP32 MFMA operands d + 2 in steps of 2;
// the FP64 operator d + 2 in steps of 4; the padded size is a multiple of
// 256 and at least n.
// The wide sweep's tiled schedule, decoded as the kernel decodes it (work
// group w: XCD w mod 8, tile (w / 8 / 32) * 8 + w mod 8, item (w / 8) mod 32
// of the tile): every pair (I, u) with 0 <= u < ndel(I) taken by exactly one
// item, every row-partial slot (I, c < nchunk) written by exactly one item,
// every column-partial slot (J, u - 1) that the reduction reads written by
// exactly one pair, and the partial buffer large enough.
static long wide_plans() {
  long count = 0;
  for (int64_t n_pad = 256; n_pad <= (int64_t(1) << 21); n_pad = n_pad * 5 / 4 / 256 * 256 + 256) {
    const int nb = static_cast<int>(n_pad / 256);
    for (int items = kSweepItemsMin; items <= kSweepItemsMax; items *= 2) {
      const MatvecPlan p = wide_plan(n_pad, items);
      CHECK(p.blk == 256 && p.nb == nb && p.dmax == nb / 2);
      CHECK(p.nchunk % 4 == 0 && p.chunk >= 1 && p.grid % 256 == 0);
      const int parts = p.nchunk / 4, S = wide_steps(nb);
      CHECK(int64_t(parts) * p.chunk >= S && int64_t(parts - 1) * p.chunk < S);
      CHECK(size_t(2 * p.nchunk + p.dmax) * size_t(n_pad) <= wide_partial_floats(n_pad));
      const int64_t tiles = int64_t((nb + kWideGroup - 1) / kWideGroup) * parts;
      std::vector<int> pair(size_t(nb) * (p.dmax + 1), 0), slot(size_t(nb) * p.nchunk, 0);
      std::vector<int> col(size_t(nb) * (p.dmax + 1), 0);
      for (int64_t w = 0; w < p.grid; ++w) {
        const int64_t j = w >> 3, tile = (j >> 5) * 8 + (w & 7);
        if (tile >= tiles) continue;
        const int grp = static_cast<int>(tile / parts), part = static_cast<int>(tile % parts);
        const int ia = static_cast<int>((j & 31) >> 2), ib = static_cast<int>(j & 3);
        const int I = kWideGroup * grp + ia;
        if (I >= nb) continue;
        const int ndel = ((nb % 2) == 0 && I >= nb / 2) ? p.dmax : p.dmax + 1;
        slot[size_t(I) * p.nchunk + 4 * part + ib] += 1;
        for (int st = part * p.chunk; st < std::min(S, (part + 1) * p.chunk); ++st) {
          const int u = 4 * st + ib - ia;
          if (u < 0 || u >= ndel) continue;
          pair[size_t(I) * (p.dmax + 1) + u] += 1;
          if (u >= 1) col[size_t((I + u) % nb) * (p.dmax + 1) + u] += 1;
        }
      }
      for (int I = 0; I < nb; ++I) {
        const int ndel = ((nb % 2) == 0 && I >= nb / 2) ? p.dmax : p.dmax + 1;
        for (int u = 0; u <= p.dmax; ++u) CHECK(pair[size_t(I) * (p.dmax + 1) + u] == (u < ndel ? 1 : 0));
        for (int c = 0; c < p.nchunk; ++c) CHECK(slot[size_t(I) * p.nchunk + c] == 1);
        // the reduction reads offsets 1 .. dlim(J) of column block J
        const int dlim = ((nb % 2) == 0 && I < nb / 2) ? p.dmax - 1 : p.dmax;
        for (int u = 1; u <= p.dmax; ++u) CHECK(col[size_t(I) * (p.dmax + 1) + u] == (u <= dlim ? 1 : 0));
      }
      ++count;
    }
  }
  return count;
}

static long geometry() {
  long count = 0;
  for (int prec = 0; prec <= 5; ++prec)
    for (int d = 1; d <= 64; ++d)
      for (int64_t n : {1, 255, 256, 257, 65536, 1000003}) {
        const Geometry g = make_geometry(n, d, prec);
        CHECK(g.n == n && g.d == d && g.prec == prec);
        CHECK(g.n_pad >= n && g.n_pad % 256 == 0 && g.n_pad - n < 256);
        if (prec == 3 || prec == 5) {
          CHECK(g.ksteps == 0);
        } else if (prec == 1 || prec == 4) {
          CHECK(g.kstride == 16 * g.ksteps && g.kstride >= d + 6);
        } else if (prec == 2) {
          CHECK(g.ksteps > 0 && 16 * g.ksteps >= 4 * d + 6);
        } else if (g.opk == kOpBf16Acc64) {
          CHECK(g.ksteps > 0 && 16 * g.ksteps >= 6 * d + 6);
        } else {
          CHECK(g.opk == kOpF32 && g.ksteps > 0 && 2 * g.ksteps >= d + 2 &&
                g.kstride >= 2 * g.ksteps);
        }
        const int ks = exact_ksteps(d);
        CHECK(4 * ks >= d + 2 && exact_stride(d) >= 4 * ks);
        ++count;
      }
  return count;
}

int main() {
  std::cout.precision(17);
  std::string cmd;
  while (std::cin >> cmd) {
    if (cmd == "plans") {
      std::cout << "plans ok " << plans() << "\n";
    } else if (cmd == "wide") {
      std::cout << "wide ok " << wide_plans() << "\n";
    } else if (cmd == "geometry") {
      std::cout << "geometry ok " << geometry() << "\n";
    } else if (cmd == "tridiag") {
      int m;
      std::cin >> m;
      std::vector<double> d(m), e(m > 0 ? m - 1 : 0), q;
      for (auto &v : d) std::cin >> v;
      for (auto &v : e) std::cin >> v;
      const bool ok = tridiag_eig_first_row(d, e, q);
      std::cout << "tridiag " << (ok ? 1 : 0);
      for (int i = 0; i < m; ++i) std::cout << " " << d[i];
      for (int i = 0; i < m; ++i) std::cout << " " << q[i];
      std::cout << "\n";
    } else if (cmd == "slq") {
      int m;
      double z2;
      std::cin >> m >> z2;
      std::vector<double> a(m), b(m > 0 ? m - 1 : 0);
      for (auto &v : a) std::cin >> v;
      for (auto &v : b) std::cin >> v;
      double out = 0.0;
      const int st = slq_quadrature(a.data(), b.data(), m, z2, &out);
      std::cout << "slq " << st << " " << out << "\n";
    } else {
      std::fprintf(stderr, "unknown command %s\n", cmd.c_str());
      return 2;
    }
  }
  return 0;
}
