// af_hier.cpp -- host quadtree of equal-size patches (Sec. 3).
//
// A hierarchy is a leaf set of the forest of quadtrees rooted at the
// n0x x n0y level-0 patches of a periodic rectangle.  Patch (l, ix, iy) of
// level l covers cells [ix m, (ix+1) m) x [iy m, (iy+1) m) of level l; its
// children are (l+1, 2ix+qx, 2iy+qy).  Lookups go through dense per-level
// tables (leaf id or -1), so every query is O(levels).
#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "af_hier.h"

namespace af {

namespace {
long long wrapi(long long v, long long n) { return ((v % n) + n) % n; }
}  // namespace

int Hier::npx(int l) const { return n0x << l; }
int Hier::npy(int l) const { return n0y << l; }

int Hier::find(int l, long long px, long long py) const {
  if (l < 0 || l > lmax) return -1;
  const long long nx = npx(l), ny = npy(l);
  px = wrapi(px, nx);
  py = wrapi(py, ny);
  return lut[size_t(lut_off[l] + py * nx + px)];
}

// Leaf covering patch position (l, px, py): the position itself or an
// ancestor; returns its id and level, or -1 if the position is subdivided.
int Hier::cover(int l, long long px, long long py, int* lev) const {
  for (int k = l; k >= 0; --k) {
    const int id = find(k, px >> (l - k), py >> (l - k));
    if (id >= 0) {
      *lev = k;
      return id;
    }
    // positions are wrapped per level inside find; shifting a wrapped value
    // stays consistent because every level's extent is a multiple of 2
  }
  return -1;
}

std::string Hier::build(const std::vector<Leaf>& in) {
  leaves = in;
  const int n = int(leaves.size());
  if (n == 0) return "empty leaf set";
  lut_off.assign(lmax + 2, 0);
  long long total = 0;
  for (int l = 0; l <= lmax; ++l) {
    lut_off[l] = int(total);
    total += (long long)npx(l) * npy(l);
  }
  lut_off[lmax + 1] = int(total);
  if (total > (1LL << 28)) return "lookup tables too large (lmax too high)";
  lut.assign(size_t(total), -1);
  level_first.assign(lmax + 2, -1);
  level_count.assign(lmax + 2, 0);
  int prev_level = -1;
  for (int k = 0; k < n; ++k) {
    const Leaf& L = leaves[k];
    if (L.level < 0 || L.level > lmax) return "leaf level out of range";
    if (L.ix < 0 || L.ix >= npx(L.level) || L.iy < 0 || L.iy >= npy(L.level)) return "leaf index out of range";
    if (L.level < prev_level) return "leaves must be sorted by level";
    prev_level = L.level;
    int& slot = lut[size_t(lut_off[L.level] + (long long)L.iy * npx(L.level) + L.ix)];
    if (slot >= 0) return "duplicate leaf";
    slot = k;
    if (level_first[L.level] < 0) level_first[L.level] = k;
    level_count[L.level]++;
  }
  // exact tiling: no leaf has a leaf ancestor, and the areas add up
  long long area = 0;
  for (const Leaf& L : leaves) {
    area += 1LL << (2 * (lmax - L.level));
    for (int k = L.level - 1; k >= 0; --k)
      if (find(k, L.ix >> (L.level - k), L.iy >> (L.level - k)) >= 0) return "leaf overlaps an ancestor leaf";
  }
  if (area != (long long)n0x * n0y << (2 * lmax)) return "leaves do not cover the domain";
  // 2:1 balance across edges and corners (periodic): the level-l positions
  // around every leaf must be covered by leaves of level >= l-1
  for (const Leaf& L : leaves)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        if (!dx && !dy) continue;
        int lev;
        if (cover(L.level, L.ix + dx, L.iy + dy, &lev) >= 0 && lev < L.level - 1)
          return "hierarchy is not 2:1 balanced";
      }
  // side relations
  rel.assign(size_t(n) * 4, 0);
  side_mask.assign(n, 0);
  static const int sdx[4] = {-1, 1, 0, 0}, sdy[4] = {0, 0, -1, 1};
  for (int k = 0; k < n; ++k) {
    const Leaf& L = leaves[k];
    for (int s = 0; s < 4; ++s) {
      const long long px = L.ix + sdx[s], py = L.iy + sdy[s];
      int r;
      if (find(L.level, px, py) >= 0) r = 0;
      else if (L.level > 0 && find(L.level - 1, wrapi(px, npx(L.level)) >> 1, wrapi(py, npy(L.level)) >> 1) >= 0) r = -1;
      else r = 1;
      rel[size_t(k) * 4 + s] = int8_t(r);
      if (r != 0) side_mask[k] |= uint8_t(1 << s);
    }
  }
  // coarse-fine faces per coarse level, grouped by coarse cell
  faces.assign(lmax + 1, {});
  for (int k = 0; k < n; ++k) {
    const Leaf& C = leaves[k];
    for (int s = 0; s < 4; ++s) {
      if (rel[size_t(k) * 4 + s] != 1) continue;
      for (int t = 0; t < m; ++t) {
        CFFace F;
        F.coarse = k;
        F.side = s;
        F.k = t;
        // the two fine faces facing coarse face t: fine index 2 (base + t)
        const long long base = (s < 2) ? (long long)C.iy * m : (long long)C.ix * m;
        const long long f0 = 2 * (base + t);
        long long fpx, fpy;
        if (s < 2) {
          fpx = (s == 0) ? 2LL * C.ix - 1 : 2LL * C.ix + 2;
          fpy = f0 / m;
        } else {
          fpy = (s == 2) ? 2LL * C.iy - 1 : 2LL * C.iy + 2;
          fpx = f0 / m;
        }
        F.fine = find(C.level + 1, fpx, fpy);
        if (F.fine < 0) return "internal: missing fine neighbour";
        F.fk = int(f0 - (f0 / m) * m);
        faces[C.level].push_back(F);
      }
    }
  }
  for (auto& fl : faces) {
    auto cell = [&](const CFFace& F) {
      const int ci = F.side == 0 ? 0 : (F.side == 1 ? m - 1 : F.k);
      const int cj = F.side == 2 ? 0 : (F.side == 3 ? m - 1 : F.k);
      return std::make_tuple(F.coarse, cj, ci, F.side);
    };
    std::stable_sort(fl.begin(), fl.end(), [&](const CFFace& a, const CFFace& b) { return cell(a) < cell(b); });
  }
  finest = 0;
  for (const Leaf& L : leaves) finest = std::max(finest, L.level);
  return "";
}

// Regrid (Sec. 3): refine tagged leaves, close under 2:1 corner balance,
// coarsen qualifying families, sort by (level, iy, ix).
std::vector<Leaf> Hier::regrid(const int8_t* tags) const {
  // the candidate leaf set as dense per-level flags, indexed like the lookup
  // table; scanning them level by level, row by row gives the (level, iy, ix)
  // order of the result
  const size_t total = lut.size();
  auto at = [&](int l, long long px, long long py) {
    const long long nx = npx(l), ny = npy(l);
    return size_t(lut_off[l] + wrapi(py, ny) * nx + wrapi(px, nx));
  };
  std::vector<uint8_t> cur(total, 0), was(total, 0);
  std::vector<int8_t> old_tag(total, 0);
  for (size_t k = 0; k < leaves.size(); ++k) {
    const Leaf& L = leaves[k];
    const size_t e = at(L.level, L.ix, L.iy);
    was[e] = 1;
    old_tag[e] = tags[k];
    if (tags[k] == 1 && L.level < lmax) {
      for (int q = 0; q < 4; ++q) cur[at(L.level + 1, 2 * L.ix + (q & 1), 2 * L.iy + (q >> 1))] = 1;
    } else {
      cur[e] = 1;
    }
  }
  // leaf of the set covering position (l, px, py), itself or an ancestor
  auto covering = [&](int l, long long px, long long py, int* lev) -> bool {
    for (int k = l; k >= 0; --k)
      if (cur[at(k, px >> (l - k), py >> (l - k))]) {
        *lev = k;
        return true;
      }
    return false;
  };
  // every leaf of the set, in (level, iy, ix) order
  auto for_each = [&](auto&& f) {
    for (int l = 0; l <= lmax; ++l)
      for (int iy = 0; iy < npy(l); ++iy)
        for (int ix = 0; ix < npx(l); ++ix)
          if (cur[size_t(lut_off[l] + (long long)iy * npx(l) + ix)]) f(l, ix, iy);
  };
  // balance closure: a leaf two levels coarser than a touching leaf splits
  std::vector<uint8_t> mark(total, 0);
  std::vector<Leaf> split;
  for (;;) {
    split.clear();
    for_each([&](int l, int ix, int iy) {
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if (!dx && !dy) continue;
          const long long px = wrapi(ix + dx, npx(l)), py = wrapi(iy + dy, npy(l));
          int lev;
          if (covering(l, px, py, &lev) && lev <= l - 2) {
            const Leaf S{lev, int(px >> (l - lev)), int(py >> (l - lev))};
            uint8_t& m = mark[at(S.level, S.ix, S.iy)];
            if (!m) {
              m = 1;
              split.push_back(S);
            }
          }
        }
    });
    if (split.empty()) break;
    for (const Leaf& S : split) {
      const size_t e = at(S.level, S.ix, S.iy);
      mark[e] = 0;
      cur[e] = 0;
      for (int q = 0; q < 4; ++q) cur[at(S.level + 1, 2 * S.ix + (q & 1), 2 * S.iy + (q >> 1))] = 1;
    }
  }
  // families: all four siblings are leaves tagged -1, and no sibling has a
  // subdivided level-l neighbour position outside the family
  std::vector<Leaf> parents;
  for_each([&](int l, int ix, int iy) {
    if (l == 0 || (ix & 1) || (iy & 1)) return;
    bool ok = true;
    for (int q = 0; q < 4 && ok; ++q) {
      const size_t e = at(l, ix + (q & 1), iy + (q >> 1));
      if (!cur[e] || !was[e] || old_tag[e] != -1) ok = false;
    }
    for (int q = 0; q < 4 && ok; ++q) {
      const int sx = ix + (q & 1), sy = iy + (q >> 1);
      for (int dy = -1; dy <= 1 && ok; ++dy)
        for (int dx = -1; dx <= 1 && ok; ++dx) {
          if (!dx && !dy) continue;
          int lev;
          if (!covering(l, wrapi(sx + dx, npx(l)), wrapi(sy + dy, npy(l)), &lev)) ok = false;  // finer leaves touch the parent
        }
    }
    if (ok) parents.push_back({l - 1, ix >> 1, iy >> 1});
  });
  for (const Leaf& P : parents) {
    for (int q = 0; q < 4; ++q) cur[at(P.level + 1, 2 * P.ix + (q & 1), 2 * P.iy + (q >> 1))] = 0;
    cur[at(P.level, P.ix, P.iy)] = 1;
  }
  std::vector<Leaf> out;
  for_each([&](int l, int ix, int iy) { out.push_back({l, ix, iy}); });
  return out;
}

}  // namespace af
