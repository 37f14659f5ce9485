// Host-side launch entry points of the device kernels (one definition per
// translation unit; the C ABI in hfx_capi.cpp calls these).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hfx_common.hpp"

namespace hfx {

// One class-segment launch over a fused quartet list.
struct SegLaunch {
  const DevSys *sys;            // device array of nsys plan descriptors
  int nsys;
  const int64_t *seg;           // device: nsys + 1 segment bounds of this class
  const uint64_t *list;         // fused quartet list
  unsigned long long *nprim;    // device counter of primitive quartets (this class)
  int64_t nq_hint;              // quartets if known on the host, -1 if not
  hipStream_t stream;
  int64_t max_blocks = 0;       // grid cap (0: the launcher's default)
};
// grid of a launch: `need` blocks if known (> 0), capped at max_blocks or def
inline int64_t seg_grid(const SegLaunch &L, int64_t need, int64_t def) {
  const int64_t cap = L.max_blocks > 0 ? L.max_blocks : def;
  return (need > 0 && need < cap) ? need : cap;
}

#define HFX_DECL_R(CB, CK)                                                                             \
  void launch_eri_r##CB##CK(int op, const SegLaunch &L);
HFX_DECL_R(0, 0)
HFX_DECL_R(1, 0)
HFX_DECL_R(1, 1)
HFX_DECL_R(2, 0)
HFX_DECL_R(2, 1)
HFX_DECL_R(2, 2)
HFX_DECL_R(3, 0)
HFX_DECL_R(3, 1)
HFX_DECL_R(3, 2)
HFX_DECL_R(3, 3)
HFX_DECL_R(4, 0)
HFX_DECL_R(4, 1)
HFX_DECL_R(4, 2)
HFX_DECL_R(4, 3)
HFX_DECL_R(5, 0)
HFX_DECL_R(5, 1)
#undef HFX_DECL_R
#define HFX_DECL_F32(CB, CK)                                                                           \
  void launch_eri_f32_r##CB##CK(int op, const SegLaunch &L);
HFX_DECL_F32(0, 0)
HFX_DECL_F32(1, 0)
HFX_DECL_F32(1, 1)
HFX_DECL_F32(2, 0)
HFX_DECL_F32(2, 1)
HFX_DECL_F32(2, 2)
HFX_DECL_F32(3, 0)
HFX_DECL_F32(3, 1)
HFX_DECL_F32(3, 2)
HFX_DECL_F32(3, 3)
HFX_DECL_F32(4, 0)
HFX_DECL_F32(4, 1)
HFX_DECL_F32(4, 2)
HFX_DECL_F32(4, 3)
HFX_DECL_F32(5, 0)
HFX_DECL_F32(5, 1)
#undef HFX_DECL_F32
void launch_schwarz_c0(int op, const DevSys &s, int p0, int p1, hipStream_t st);
void launch_schwarz_c1(int op, const DevSys &s, int p0, int p1, hipStream_t st);
void launch_schwarz_c2(int op, const DevSys &s, int p0, int p1, hipStream_t st);
void launch_schwarz_c3(int op, const DevSys &s, int p0, int p1, hipStream_t st);


// classes evaluated only by the cooperative kernels (their one-lane recursion
// would spill): (dp|dp), (dd|pp), (dd|ds), (dd|dp), (dd|dd)
__host__ __device__ constexpr bool register_available(int cb, int ck) {
  return !((cb == 4 && ck == 4) || (cb == 5 && ck >= 2));
}
void launch_eri(int cb, int ck, int op, const SegLaunch &L);
void launch_eri_f32(int cb, int ck, int op, const SegLaunch &L);

// lane-per-component kernels (FP64 and FP32) of the classes whose bra pair
// is pp or has a d shell
__host__ __device__ constexpr bool lane_available(int cb, int ck) { return cb >= 2 && ck <= cb; }
struct CoopDev;
void launch_eri_lane(int cb, int ck, int op, bool f32, const CoopDev &cd, const SegLaunch &L);
// doubles of HRR workspace the lane kernel of the class reserves
int lane_hrr_capacity(int cb, int ck);
void launch_schwarz(int cb, int op, const DevSys &s, int p0, int p1, hipStream_t st);
void launch_zero_i32(int32_t *p, int64_t n, hipStream_t st);

// D (boundary basis) -> D_cart and P_max per block (canonical block decides,
// partner copies); global max into s.pmax_global.  accumulate: P_max becomes
// the larger of its current value and this density's (second spin).
void launch_density(const DevSys &s, int64_t nblk, const int2 *blk_IJ, const int64_t *blk_off,
                    const int32_t *partner, const uint8_t *canon, int spherical, const double *D, double *Dc,
                    bool accumulate, hipStream_t st);
// K_cart = K4 + K4^T (image flip), K = T K_cart T^T written in the boundary basis.
void launch_finalize(const DevSys &s, int64_t nblk, const int2 *blk_IJ, const int64_t *blk_off,
                     const int32_t *partner, int spherical, const double *K4, double *K, hipStream_t st);
void launch_zero(double *p, int64_t n, hipStream_t st);
// H(k) = scale sum_G K^G exp(i k.(T_G + r_J - r_I)), dense complex [nk][nbf][nbf]
// (zeroed first); pairs: (I, J, first pattern block, block count) of every
// shell pair of the pattern; blk_img: packed image (8 bits per component)
// of each block; func_off: first boundary function of each shell.
void launch_kspace(const DevSys &s, const int4 *pairs, int npairs, const int32_t *blk_img, const int64_t *blk_off,
                   const int32_t *func_off, int sph, const double *K, const double *kpts, int nk, int64_t nbf,
                   double scale, double *H, hipStream_t st);
void launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t st);
// Screening over fused work items (region, bra pair, plan), one wave per
// item.  mode: 0 every kept quartet, 1 only Q_IJ*Q_KL >= the region's
// fp32_cut (FP64 list), 2 only Q_IJ*Q_KL < fp32_cut (FP32 list).  Count pass
// writes counts[item]; fill pass writes item's quartets at offsets[item] -
// base and never at or beyond cap (sets err bit 2).  A chunk of the list is
// filled by passing the chunk's first item (items + i0, offsets + i0), its
// item count and base = offsets[i0].
void launch_screen(const DevSys *sys, const int4 *items, int64_t nitems, int32_t *counts, const int64_t *offsets,
                   uint64_t *out, int64_t base, int64_t cap, int32_t *err, bool fill, int mode, hipStream_t st);
// seg[k] = clamp(offsets[seg_items[k]], lo, hi) - lo, k < n: class-segment
// bounds on the device of the list part [lo, hi) held in the list buffer
// (lo = 0, hi = capacity for a whole list: a replayed graph whose screened
// count overflows never reads past the list)
void launch_gather_bounds(const int64_t *offsets, const int64_t *seg_items, int64_t *seg, int n, int64_t lo,
                          int64_t hi, hipStream_t st);
// exclusive prefix sum of int32 counts into int64 offsets (n+1 entries)
// tiles: device scratch of at least (n + 1023) / 1024 entries
hipError_t scan_counts(const int32_t *counts, int64_t *offsets, int64_t n, int64_t *tiles, hipStream_t st);

}  // namespace hfx
