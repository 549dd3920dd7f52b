// af_hier.h -- host quadtree (Sec. 3).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "af_internal.h"

namespace af {

struct Leaf {
  int level, ix, iy;
};

struct Hier {
  int m = 16, n0x = 1, n0y = 1, lmax = 0;
  std::vector<Leaf> leaves;
  std::vector<int32_t> lut;       // dense per-level leaf ids
  std::vector<int> lut_off;       // [lmax+2]
  std::vector<int> level_first, level_count;
  std::vector<int8_t> rel;        // [n][4] side relations
  std::vector<uint8_t> side_mask; // [n]
  std::vector<std::vector<CFFace>> faces;  // per coarse level
  int finest = 0;

  int npx(int l) const;
  int npy(int l) const;
  int find(int l, long long px, long long py) const;
  int cover(int l, long long px, long long py, int* lev) const;
  // builds all tables; returns an error message or "" on success
  std::string build(const std::vector<Leaf>& in);
  std::vector<Leaf> regrid(const int8_t* tags) const;
};

}  // namespace af
