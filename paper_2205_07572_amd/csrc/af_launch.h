// af_launch.h -- host-side launch descriptors of the library's kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "af_internal.h"

namespace af {

struct StepLaunch {
  bool fp32;
  int eq, m, ty;
  const void* in[4];
  void* out[4];
  int npatch, pitch, first, count, region;
  double dtdx, dtdy, a, b, c;
  double len_dt_x, len_dt_y;
  double* reg;
  const uint8_t* side_mask;
  const int32_t* leaf_xy;  // [npatch][2] patch (ix, iy); rotation only
  const void* weights;  // AdvWeights<T>, AcWeights<T> or RotParams<T> matching fp32/eq
  int gnx = 0, gny = 0;  // > 0: complete level, cells outside a patch come from its neighbours
};

struct AdvanceLaunch {
  bool fp32;
  int eq, m, k, nt;
  const void* in[4];
  void* out[4];
  int npatch, pitch, first, count;
  int nx, ny;  // patches per side of the (complete, row-major) level
  double dtdx, dtdy, a, b, c;
  const void* weights;
};

struct BufLaunch {
  void* p[2][4];
  int npatch, pitch, m, ncomp;
  uint32_t mask;
};

// One time point of the batched subcycled coarse step (constant-coefficient
// equations): levels lev0 .. lev0 + nlev - 1 step together; level lev0 + k
// holds leaves [first[k], first[k] + count[k]) and steps `region[k]`.
struct AmrStepLaunch {
  bool fp32;
  int eq, m, ty;
  void* p[2][4];
  int npatch, pitch;
  uint32_t mask;
  int nlev, lev0;
  int first[kMaxLevels], count[kMaxLevels], region[kMaxLevels];
  double len_dt_x[kMaxLevels], len_dt_y[kMaxLevels];
  double dtdx, dtdy, a, b, c;
  double* reg;
  const uint8_t* side_mask;
  const int4* plan;
  const int32_t* entries;
  int nentries, ninner;
  const FillWeights* fw;
  const int32_t* nbr;
  const uint32_t* gnflags;
  const void* weights;  // AdvWeights<T> or AcAllWeights<T>
  const void* weights_dev;  // acoustics: AcOrbitWeights<T> on the device
  // the last level (the finest, region layer 1) takes both substeps of its
  // pair in one block (m = 8 or 16; whole-patch tiles)
  bool pair;
};
// m for which a fused pair of finest-level substeps is compiled
inline bool amr_pair_supported(int m) { return m == 8 || m == 16; }
hipError_t launch_amr_step(const AmrStepLaunch& s, hipStream_t st);

// Conservative fix of faces [0, nfaces) and the fill's vertex copies onto
// the closed-square boundary nodes of the leaves canon[0 .. ncanon).
struct AmrSyncLaunch {
  bool fp32;
  BufLaunch b;
  const int32_t* plevel;
  const int4* cops;  // vertex copies (launch_canon_ops)
  int ncops;
  const CFFace* faces;
  int nfaces;
  double* reg;
  double inv_area0;
};
hipError_t launch_amr_sync(const AmrSyncLaunch& s, hipStream_t st);
// Resolves the vertex copies of the leaves canon[0 .. ncanon) (boundary
// entries bnd of the fill set) from the fill plan into ncanon * nbnd ops.
hipError_t launch_canon_ops(const int4* plan, const int32_t* entries, int nentries, const int32_t* bnd, int nbnd,
                            const int32_t* canon, int ncanon, const int32_t* plevel, int4* ops, hipStream_t st);

hipError_t launch_patch_step(const StepLaunch& s, hipStream_t st);
hipError_t launch_level_advance(const AdvanceLaunch& s, hipStream_t st);
// Fills the level-advance shapes (K, threads) for (precision, equation, m) and
// returns their count.  With up, also the shapes only the upwind one-pass
// kernel runs.
int level_advance_shapes(bool fp32, int eq, int m, int* ks, int* nts, int cap, bool up);
// Whether advection weights take every node from the upwind source pattern
// (false for acoustics).
bool level_advance_up_pattern(bool fp32, int eq, const void* weights);
// nblocks x kThreads threads, 8 chains x 16 x iters FMAs each
hipError_t launch_fma_probe(bool fp32, void* out, int nblocks, int iters, hipStream_t st);
bool step_shape_supported(int m, int ty);
// resolves the fill sources of every leaf (sources of level >= smin) into
// plan[nleaves][nentries] and flags[nleaves] (bit p: ops of phase p); with
// nbr and gnflags non-null also the same-level neighbours [nleaves][9] and
// the directions a same-level gather stages (bit d)
hipError_t launch_fill_plan(const HierDev& H, const int32_t* entries, int nentries, int m, int smin, int4* plan,
                            uint32_t* flags, int32_t* nbr, uint32_t* gnflags, hipStream_t st);
// applies the phase-`phase` ops of leaves [first_target, first_target + ntargets)
hipError_t launch_fill_apply(bool fp32, const BufLaunch& b, const HierDev& H, const int32_t* entries, int nentries,
                             const int4* plan, const uint32_t* flags, const FillWeights* W, int first_target,
                             int ntargets, int phase, hipStream_t st);
hipError_t launch_flux_correct(bool fp32, const BufLaunch& b, const CFFace* faces, int nfaces, double* reg,
                               int level, double inv_area, hipStream_t st);
hipError_t launch_tag(bool fp32, const BufLaunch& b, const HierDev& H, int mode, int comp, double inv2dx0,
                      double inv2dy0, double tr, double tc, int8_t* tags, double* values, hipStream_t st);
hipError_t launch_transfer(bool fp32, const BufLaunch& old_b, const HierDev& HO, const BufLaunch& new_b,
                           const Transfer* tr, int nnew, hipStream_t st);
// Capacity (doubles) of the statically allocated partial-sum scratch of
// af_reduce_sum_noalloc: nleaves * ncomp partial sums.
constexpr size_t kScratchSums = size_t(3) * 65536;
// The calling thread's current device's address of that scratch (looked up
// on the first call per device).
hipError_t scratch_sums(double** ptr);
hipError_t launch_sum(bool fp32, const BufLaunch& b, const HierDev& H, double area0, double* part, double* out,
                      hipStream_t st);

}  // namespace af
