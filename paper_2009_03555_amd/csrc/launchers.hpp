// Host-side launch entry points of the device kernels (one definition per
// translation unit; the C ABI in hfx_capi.cpp calls these).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hfx_common.hpp"

namespace hfx {

#define HFX_DECL_R(CB, CK)                                                                             \
  void launch_eri_r##CB##CK(int op, const DevSys &s, const uint64_t *list, int64_t nq, const double *Dc,  \
                            double *K4, unsigned long long *nprim, hipStream_t st);
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
HFX_DECL_R(4, 4)
HFX_DECL_R(5, 0)
HFX_DECL_R(5, 1)
HFX_DECL_R(5, 2)
HFX_DECL_R(5, 3)
HFX_DECL_R(5, 4)
HFX_DECL_R(5, 5)
#undef HFX_DECL_R
void launch_schwarz_c0(int op, const DevSys &s, int p0, int p1, hipStream_t st);
void launch_schwarz_c1(int op, const DevSys &s, int p0, int p1, hipStream_t st);
void launch_schwarz_c2(int op, const DevSys &s, int p0, int p1, hipStream_t st);
void launch_schwarz_c3(int op, const DevSys &s, int p0, int p1, hipStream_t st);
void launch_schwarz_c4(int op, const DevSys &s, int p0, int p1, hipStream_t st);
void launch_schwarz_c5(int op, const DevSys &s, int p0, int p1, hipStream_t st);


void launch_eri(int cb, int ck, int op, const DevSys &s, const uint64_t *list, int64_t nq, const double *Dc,
                double *K4, unsigned long long *nprim, hipStream_t st);
void launch_schwarz(int cb, int op, const DevSys &s, int p0, int p1, hipStream_t st);

// D (boundary basis) -> D_cart and P_max per block (canonical block decides,
// partner copies); global max into s.pmax_global.
void launch_density(const DevSys &s, int64_t nblk, const int2 *blk_IJ, const int64_t *blk_off,
                    const int32_t *partner, const uint8_t *canon, int spherical, const double *D, double *Dc,
                    hipStream_t st);
// K_cart = K4 + K4^T (image flip), K = T K_cart T^T written in the boundary basis.
void launch_finalize(const DevSys &s, int64_t nblk, const int2 *blk_IJ, const int64_t *blk_off,
                     const int32_t *partner, int spherical, const double *K4, double *K, hipStream_t st);
void launch_zero(double *p, int64_t n, hipStream_t st);
void launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t st);
// Screening: one wave per item (region, bra pair).  count pass writes
// counts[item]; fill pass writes the quartets at offsets[item].
void launch_screen(const DevSys &s, const int2 *items, int64_t nitems, const int32_t *class_start,
                   int32_t *counts, const int64_t *offsets, uint64_t *out, int32_t *err, bool fill,
                   hipStream_t st);
// exclusive prefix sum of int32 counts into int64 offsets (n+1 entries)
hipError_t scan_counts(const int32_t *counts, int64_t *offsets, int64_t n, void *tmp, size_t &tmp_bytes,
                       hipStream_t st);

}  // namespace hfx
