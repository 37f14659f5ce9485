// Bandwidth-bound kernels around the ERI phase: density transform and
// P_max (Eq. dmscreening), quartet screening and compaction (Eq. schwarz
// times P_scr, 8-fold unique enumeration), K finalisation, fills.

#include <cstdlib>

#include "coop.hpp"
#include "launchers.hpp"

namespace hfx {

// --------------------------------------------------------- dispatchers
void launch_eri(int cb, int ck, int op, const SegLaunch &L) {
  typedef void (*fn)(int, const SegLaunch &);
  static const fn table[kNQuartetClass] = {
      launch_eri_r00, launch_eri_r10, launch_eri_r11, launch_eri_r20, launch_eri_r21, launch_eri_r22,
      launch_eri_r30, launch_eri_r31, launch_eri_r32, launch_eri_r33, launch_eri_r40, launch_eri_r41,
      launch_eri_r42, launch_eri_r43, nullptr, launch_eri_r50, launch_eri_r51, nullptr,
      nullptr, nullptr, nullptr};
  if (cb < 0 || cb >= kNPairClass || ck < 0 || ck > cb || !table[region_of(cb, ck)]) return;
  table[region_of(cb, ck)](op, L);
}

void launch_eri_coop_r42(int op, const CoopDev &cd, const SegLaunch &L);
void launch_eri_coop_r43(int op, const CoopDev &cd, const SegLaunch &L);
void launch_eri_coop_r44(int op, const CoopDev &cd, const SegLaunch &L);
void launch_eri_coop_r51(int op, const CoopDev &cd, const SegLaunch &L);
void launch_eri_coop_r52(int op, const CoopDev &cd, const SegLaunch &L);
void launch_eri_coop_r53(int op, const CoopDev &cd, const SegLaunch &L);
void launch_eri_coop_r54(int op, const CoopDev &cd, const SegLaunch &L);
void launch_eri_coop_r55(int op, const CoopDev &cd, const SegLaunch &L);

void launch_schwarz_coop_c4(int op, const DevSys *sys1, const CoopDev &cd, int p0, int p1, hipStream_t st);
void launch_schwarz_coop_c5(int op, const DevSys *sys1, const CoopDev &cd, int p0, int p1, hipStream_t st);
void launch_schwarz_coop(int cb, int op, const DevSys *sys1, const CoopDev &cd, int p0, int p1, hipStream_t st) {
  if (cb == 4) launch_schwarz_coop_c4(op, sys1, cd, p0, p1, st);
  if (cb == 5) launch_schwarz_coop_c5(op, sys1, cd, p0, p1, st);
}

void launch_eri_coop(int cb, int ck, int op, const CoopDev &cd, const SegLaunch &L) {
  switch (cb * 10 + ck) {
    case 42: launch_eri_coop_r42(op, cd, L); break;
    case 43: launch_eri_coop_r43(op, cd, L); break;
    case 44: launch_eri_coop_r44(op, cd, L); break;
    case 51: launch_eri_coop_r51(op, cd, L); break;
    case 52: launch_eri_coop_r52(op, cd, L); break;
    case 53: launch_eri_coop_r53(op, cd, L); break;
    case 54: launch_eri_coop_r54(op, cd, L); break;
    case 55: launch_eri_coop_r55(op, cd, L); break;
    default: break;
  }
}

void launch_eri_f32(int cb, int ck, int op, const SegLaunch &L) {
  typedef void (*fn)(int, const SegLaunch &);
  static const fn table[kNQuartetClass] = {
      launch_eri_f32_r00, launch_eri_f32_r10, launch_eri_f32_r11, launch_eri_f32_r20, launch_eri_f32_r21,
      launch_eri_f32_r22, launch_eri_f32_r30, launch_eri_f32_r31, launch_eri_f32_r32, launch_eri_f32_r33,
      launch_eri_f32_r40, launch_eri_f32_r41, launch_eri_f32_r42, launch_eri_f32_r43, nullptr,
      launch_eri_f32_r50, launch_eri_f32_r51, nullptr, nullptr, nullptr, nullptr};
  if (cb < 0 || cb >= kNPairClass || ck < 0 || ck > cb || !table[region_of(cb, ck)]) return;
  table[region_of(cb, ck)](op, L);
}

#define HFX_DECL_LANE(CB, CK)                                                                          \
  void launch_eri_lane_r##CB##CK(int op, bool f32, const CoopDev &cd, const SegLaunch &L);             \
  int lane_hrr_capacity_r##CB##CK();
HFX_DECL_LANE(2, 0)
HFX_DECL_LANE(2, 1)
HFX_DECL_LANE(2, 2)
HFX_DECL_LANE(3, 0)
HFX_DECL_LANE(3, 1)
HFX_DECL_LANE(3, 2)
HFX_DECL_LANE(3, 3)
HFX_DECL_LANE(4, 0)
HFX_DECL_LANE(4, 1)
HFX_DECL_LANE(4, 2)
HFX_DECL_LANE(4, 3)
HFX_DECL_LANE(4, 4)
HFX_DECL_LANE(5, 0)
HFX_DECL_LANE(5, 1)
HFX_DECL_LANE(5, 2)
HFX_DECL_LANE(5, 3)
HFX_DECL_LANE(5, 4)
HFX_DECL_LANE(5, 5)
#undef HFX_DECL_LANE

void launch_eri_lane(int cb, int ck, int op, bool f32, const CoopDev &cd, const SegLaunch &L) {
  switch (cb * 10 + ck) {
    case 20: launch_eri_lane_r20(op, f32, cd, L); break;
    case 21: launch_eri_lane_r21(op, f32, cd, L); break;
    case 22: launch_eri_lane_r22(op, f32, cd, L); break;
    case 30: launch_eri_lane_r30(op, f32, cd, L); break;
    case 31: launch_eri_lane_r31(op, f32, cd, L); break;
    case 32: launch_eri_lane_r32(op, f32, cd, L); break;
    case 33: launch_eri_lane_r33(op, f32, cd, L); break;
    case 40: launch_eri_lane_r40(op, f32, cd, L); break;
    case 41: launch_eri_lane_r41(op, f32, cd, L); break;
    case 42: launch_eri_lane_r42(op, f32, cd, L); break;
    case 43: launch_eri_lane_r43(op, f32, cd, L); break;
    case 44: launch_eri_lane_r44(op, f32, cd, L); break;
    case 50: launch_eri_lane_r50(op, f32, cd, L); break;
    case 51: launch_eri_lane_r51(op, f32, cd, L); break;
    case 52: launch_eri_lane_r52(op, f32, cd, L); break;
    case 53: launch_eri_lane_r53(op, f32, cd, L); break;
    case 54: launch_eri_lane_r54(op, f32, cd, L); break;
    case 55: launch_eri_lane_r55(op, f32, cd, L); break;
    default: break;
  }
}

int lane_hrr_capacity(int cb, int ck) {
  switch (cb * 10 + ck) {
    case 20: return lane_hrr_capacity_r20();
    case 21: return lane_hrr_capacity_r21();
    case 22: return lane_hrr_capacity_r22();
    case 30: return lane_hrr_capacity_r30();
    case 31: return lane_hrr_capacity_r31();
    case 32: return lane_hrr_capacity_r32();
    case 33: return lane_hrr_capacity_r33();
    case 40: return lane_hrr_capacity_r40();
    case 41: return lane_hrr_capacity_r41();
    case 42: return lane_hrr_capacity_r42();
    case 43: return lane_hrr_capacity_r43();
    case 44: return lane_hrr_capacity_r44();
    case 50: return lane_hrr_capacity_r50();
    case 51: return lane_hrr_capacity_r51();
    case 52: return lane_hrr_capacity_r52();
    case 53: return lane_hrr_capacity_r53();
    case 54: return lane_hrr_capacity_r54();
    case 55: return lane_hrr_capacity_r55();
    default: return 0;
  }
}

void launch_schwarz(int cb, int op, const DevSys &s, int p0, int p1, hipStream_t st) {
  switch (cb) {
    case 0: launch_schwarz_c0(op, s, p0, p1, st); break;
    case 1: launch_schwarz_c1(op, s, p0, p1, st); break;
    case 2: launch_schwarz_c2(op, s, p0, p1, st); break;
    case 3: launch_schwarz_c3(op, s, p0, p1, st); break;
    default: break;
  }
}

// ------------------------------------------------- spherical transform
// Rows: real solid harmonics m = -2..2; columns xx, xy, xz, yy, yz, zz.
__constant__ double kSphD[5][6] = {
    {0.0, 1.7320508075688772935, 0.0, 0.0, 0.0, 0.0},
    {0.0, 0.0, 0.0, 0.0, 1.7320508075688772935, 0.0},
    {-0.5, 0.0, 0.0, -0.5, 0.0, 1.0},
    {0.0, 0.0, 1.7320508075688772935, 0.0, 0.0, 0.0},
    {0.86602540378443864676, 0.0, 0.0, -0.86602540378443864676, 0.0, 0.0}};

__device__ __forceinline__ int nfunc_dev(int l, int sph) { return (l == 2 && sph) ? 5 : (l + 1) * (l + 2) / 2; }
// T[m][a] of shell l (identity unless spherical d)
__device__ __forceinline__ double tmat(int l, int sph, int m, int a) {
  if (l == 2 && sph) return kSphD[m][a];
  return m == a ? 1.0 : 0.0;
}

__global__ void density_kernel(DevSys s, int64_t nblk, const int2 *__restrict__ blk_IJ,
                               const int64_t *__restrict__ blk_off, const int32_t *__restrict__ partner,
                               const uint8_t *__restrict__ canon, int sph, const double *__restrict__ D,
                               double *__restrict__ Dc, int accumulate) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblk) return;
  const int2 ij = blk_IJ[b];
  const int li = s.sh_l[ij.x], lj = s.sh_l[ij.y];
  const int ni = nfunc_dev(li, sph), nj = nfunc_dev(lj, sph);
  const int ci = ncart(li), cj = ncart(lj);
  const double *src = D + blk_off[b];
  double *dst = Dc + s.blk_coff[b];
  const bool ti = (li == 2 && sph), tj = (lj == 2 && sph);
  double pm = 0.0;
  for (int a = 0; a < ci; ++a)
    for (int c = 0; c < cj; ++c) {
      double v;
      if (!ti && !tj) {
        v = src[a * nj + c];
      } else {
        v = 0.0;
        for (int m = 0; m < ni; ++m) {
          const double tma = ti ? kSphD[m][a] : (m == a ? 1.0 : 0.0);
          if (tma == 0.0) continue;
          double r = 0.0;
          for (int n = 0; n < nj; ++n) {
            const double tnc = tj ? kSphD[n][c] : (n == c ? 1.0 : 0.0);
            r += src[m * nj + n] * tnc;
          }
          v += tma * r;
        }
      }
      dst[a * cj + c] = v;
      pm = fmax(pm, fabs(v));
    }
  if (canon[b]) {
    // a second spin density keeps the larger block maximum of the two
    if (accumulate) pm = fmax(pm, s.pmax[b]);
    s.pmax[b] = pm;
    s.pmax[partner[b]] = pm;
    atomicMax(s.pmax_global, (unsigned long long)__double_as_longlong(pm));
  }
}

void launch_density(const DevSys &s, int64_t nblk, const int2 *blk_IJ, const int64_t *blk_off,
                    const int32_t *partner, const uint8_t *canon, int spherical, const double *D, double *Dc,
                    bool accumulate, hipStream_t st) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(density_kernel, dim3((unsigned)((nblk + 255) / 256)), dim3(256), 0, st, s, nblk, blk_IJ,
                     blk_off, partner, canon, spherical, D, Dc, accumulate ? 1 : 0);
}

// ------------------------------------------------------------ finalize
__global__ void finalize_kernel(DevSys s, int64_t nblk, const int2 *__restrict__ blk_IJ,
                                const int64_t *__restrict__ blk_off, const int32_t *__restrict__ partner,
                                int sph, const double *__restrict__ K4, double *__restrict__ K) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblk) return;
  const int2 ij = blk_IJ[b];
  const int li = s.sh_l[ij.x], lj = s.sh_l[ij.y];
  const int ni = nfunc_dev(li, sph), nj = nfunc_dev(lj, sph);
  const int ci = ncart(li), cj = ncart(lj);
  const double *k1 = K4 + s.blk_coff[b];
  const double *k2 = K4 + s.blk_coff[partner[b]];  // (J, I, -n): ci x cj transposed
  double kc[36];
  for (int a = 0; a < ci; ++a)
    for (int c = 0; c < cj; ++c) kc[a * cj + c] = k1[a * cj + c] + k2[c * ci + a];
  double *dst = K + blk_off[b];
  const bool ti = (li == 2 && sph), tj = (lj == 2 && sph);
  for (int m = 0; m < ni; ++m)
    for (int n = 0; n < nj; ++n) {
      double v;
      if (!ti && !tj) {
        v = kc[m * cj + n];
      } else {
        v = 0.0;
        for (int a = 0; a < ci; ++a) {
          const double tma = ti ? kSphD[m][a] : (m == a ? 1.0 : 0.0);
          if (tma == 0.0) continue;
          double r = 0.0;
          for (int c = 0; c < cj; ++c) {
            const double tnc = tj ? kSphD[n][c] : (n == c ? 1.0 : 0.0);
            r += kc[a * cj + c] * tnc;
          }
          v += tma * r;
        }
      }
      dst[m * nj + n] = v;
    }
}

void launch_finalize(const DevSys &s, int64_t nblk, const int2 *blk_IJ, const int64_t *blk_off,
                     const int32_t *partner, int spherical, const double *K4, double *K, hipStream_t st) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)((nblk + 255) / 256)), dim3(256), 0, st, s, nblk, blk_IJ,
                     blk_off, partner, spherical, K4, K);
}

// --------------------------------------------------------------- fills
__global__ void zero_kernel(double *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}
__global__ void zero_u64_kernel(unsigned long long *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}
void launch_zero(double *p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
}
void launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
}

// ----------------------------------------------------------- screening
__device__ __forceinline__ bool lex_nonneg(int a, int b, int c) {
  return a > 0 || (a == 0 && (b > 0 || (b == 0 && c >= 0)));
}

__device__ __forceinline__ double pmax_at(const DevSys &s, int I, int J, int a, int b, int c) {
  const int k = lookup(s, I, J, a, b, c);
  return k < 0 ? 0.0 : s.pmax[k];
}

// Visit every ket translation G of the quartet (p | q^G) that survives
// (Q_p * Q_q) * P_scr > tau.  For p == q only G >= 0 (lexicographic) is
// visited: (p|p^G) and (p|p^-G) are one orbit of the permutation relations.
template <typename F>
__device__ __forceinline__ void visit_kept(const DevSys &s, int p, int q, double Qp, double Qq, double pglob,
                                           int mode, double cut32, int32_t *err, F &&emit) {
  const double qq = Qp * Qq;
  if (!(qq * pglob > s.tau)) return;
  if (mode == 1 && !(qq >= cut32)) return;
  if (mode == 2 && !(qq < cut32)) return;
  const int4 bi = s.pr_info[p], ki = s.pr_info[q];
  int nB1, nB2, nB3, nD1, nD2, nD3;
  unpack_img8(bi.z, nB1, nB2, nB3);
  unpack_img8(ki.z, nD1, nD2, nD3);
  const int A = bi.x, B = bi.y, C = ki.x, D = ki.y;
  auto test = [&](int g1, int g2, int g3) {
    double ps = pmax_at(s, A, C, g1, g2, g3);
    ps = fmax(ps, pmax_at(s, A, D, g1 + nD1, g2 + nD2, g3 + nD3));
    ps = fmax(ps, pmax_at(s, B, C, g1 - nB1, g2 - nB2, g3 - nB3));
    ps = fmax(ps, pmax_at(s, B, D, g1 + nD1 - nB1, g2 + nD2 - nB2, g3 + nD3 - nB3));
    const double bound = qq * ps;
    return bound > s.tau;
  };
  if (!s.periodic) {
    if (test(0, 0, 0)) emit(0, 0, 0);
    return;
  }
  const double *gp = s.pr_geom + (int64_t)p * 8;
  const double *gq = s.pr_geom + (int64_t)q * 8;
  const double dx = gp[3] - gq[3], dy = gp[4] - gq[4], dz = gp[5] - gq[5];
  const double R = gp[6] + gq[6] + s.cutoff + 1e-6;
  int lo[3], hi[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double f = s.rec[3 * i] * dx + s.rec[3 * i + 1] * dy + s.rec[3 * i + 2] * dz;
    lo[i] = (int)ceil(f - R * s.recn[i]);
    hi[i] = (int)floor(f + R * s.recn[i]);
  }
  for (int g1 = lo[0]; g1 <= hi[0]; ++g1)
    for (int g2 = lo[1]; g2 <= hi[1]; ++g2)
      for (int g3 = lo[2]; g3 <= hi[2]; ++g3) {
        if (p == q && !lex_nonneg(g1, g2, g3)) continue;
        const double tx = g1 * s.lat[0] + g2 * s.lat[3] + g3 * s.lat[6];
        const double ty = g1 * s.lat[1] + g2 * s.lat[4] + g3 * s.lat[7];
        const double tz = g1 * s.lat[2] + g2 * s.lat[5] + g3 * s.lat[8];
        const double ex = dx - tx, ey = dy - ty, ez = dz - tz;
        if (ex * ex + ey * ey + ez * ez > R * R) continue;
        if (!test(g1, g2, g3)) continue;
        if (g1 < -16 || g1 > 15 || g2 < -16 || g2 > 15 || g3 < -16 || g3 > 15) {
          atomicOr(err, 1);
          continue;
        }
        emit(g1, g2, g3);
      }
}

__global__ __launch_bounds__(256) void screen_kernel(const DevSys *__restrict__ sys,
                                                     const int4 *__restrict__ items, int64_t nitems,
                                                     int32_t *__restrict__ counts,
                                                     const int64_t *__restrict__ offsets,
                                                     uint64_t *__restrict__ out, int64_t base, int64_t cap,
                                                     int32_t *err, int fill, int mode) {
  const int lane = threadIdx.x & 63;
  const int64_t item = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (item >= nitems) return;  // whole wave leaves together
  const int4 it = items[item];
  const int r = it.x, p = it.y;
  const DevSys &s = sys[it.z];
  const int32_t *class_start = s.class_start;
  int cb = 0;
  while ((cb + 1) * (cb + 2) / 2 <= r) ++cb;
  const int ck = r - cb * (cb + 1) / 2;
  const int q0 = class_start[ck];
  const int q1 = (cb == ck) ? p + 1 : class_start[ck + 1];
  const double Qp = s.pr_Q[p];
  const double cut32 = s.fp32_cut[r];
  const double pglob = __longlong_as_double((long long)*s.pmax_global);
  int64_t running = fill ? offsets[item] - base : 0;
  for (int qt = q0; qt < q1; qt += 64) {
    const int q = qt + lane;
    int cnt = 0;
    double Qq = 0.0;
    if (q < q1) {
      Qq = s.pr_Q[q];
      visit_kept(s, p, q, Qp, Qq, pglob, mode, cut32, err, [&](int, int, int) { ++cnt; });
    }
    // wave-wide inclusive scan of cnt
    int x = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    const int total = __shfl(x, 63, 64);
    if (fill && q < q1 && cnt) {
      int64_t pos = running + (x - cnt);
      visit_kept(s, p, q, Qp, Qq, pglob, mode, cut32, err, [&](int g1, int g2, int g3) {
        if (pos < cap)
          out[pos] = pack_quartet((uint32_t)p, (uint32_t)q, pack_img5(g1, g2, g3));
        else
          atomicOr(err, 2);
        ++pos;
      });
    }
    running += total;
  }
  if (!fill && lane == 0) counts[item] = (int32_t)running;
}

void launch_screen(const DevSys *sys, const int4 *items, int64_t nitems, int32_t *counts, const int64_t *offsets,
                   uint64_t *out, int64_t base, int64_t cap, int32_t *err, bool fill, int mode, hipStream_t st) {
  if (nitems <= 0) return;
  const int64_t blocks = (nitems + 3) / 4;
  hipLaunchKernelGGL(screen_kernel, dim3((unsigned)blocks), dim3(256), 0, st, sys, items, nitems, counts, offsets,
                     out, base, cap, err, fill ? 1 : 0, mode);
}

__global__ void gather_bounds_kernel(const int64_t *__restrict__ offsets, const int64_t *__restrict__ seg_items,
                                     int64_t *__restrict__ seg, int n, int64_t lo, int64_t hi) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) {
    int64_t v = offsets[seg_items[k]];
    v = v < lo ? lo : (v > hi ? hi : v);
    seg[k] = v - lo;
  }
}

void launch_gather_bounds(const int64_t *offsets, const int64_t *seg_items, int64_t *seg, int n, int64_t lo,
                          int64_t hi, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(gather_bounds_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, offsets, seg_items,
                     seg, n, lo, hi);
}

__global__ void zero_i32_kernel(int32_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}
void launch_zero_i32(int32_t *p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(zero_i32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
}

// Exclusive scan of int32 counts into int64 offsets (offsets[0] = 0,
// offsets[i+1] = sum_{k<=i} counts[k]) in three plain kernels: tile sums,
// scan of the tile sums, tile-local scan plus tile base.  Only kernel nodes,
// so the sequence can sit inside a captured graph.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanTile = kScanThreads * kScanPer;

__device__ __forceinline__ int64_t block_incl_scan(int64_t v, int64_t *sh, int64_t *total = nullptr) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = 1; d < kScanThreads; d <<= 1) {
    const int64_t add = t >= d ? sh[t - d] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  const int64_t r = sh[t];
  if (total) *total = sh[kScanThreads - 1];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kScanThreads) void scan_tile_sums(const int32_t *__restrict__ counts, int64_t n,
                                                                int64_t *__restrict__ tiles) {
  __shared__ int64_t sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  int64_t v = 0;
  for (int k = 0; k < kScanPer; ++k)
    if (base + k < n) v += counts[base + k];
  const int64_t incl = block_incl_scan(v, sh);
  if (threadIdx.x == kScanThreads - 1) tiles[blockIdx.x] = incl;
}

// one block: exclusive scan of the tile sums in place
__global__ __launch_bounds__(kScanThreads) void scan_tiles(int64_t *__restrict__ tiles, int64_t ntiles) {
  __shared__ int64_t sh[kScanThreads];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < ntiles; b0 += kScanThreads) {
    const int64_t i = b0 + threadIdx.x;
    const int64_t v = i < ntiles ? tiles[i] : 0;
    int64_t tot;
    const int64_t incl = block_incl_scan(v, sh, &tot);
    if (i < ntiles) tiles[i] = carry + incl - v;
    carry += tot;
  }
}

__global__ __launch_bounds__(kScanThreads) void scan_apply(const int32_t *__restrict__ counts, int64_t n,
                                                            const int64_t *__restrict__ tiles,
                                                            int64_t *__restrict__ offsets) {
  __shared__ int64_t sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  int64_t c[kScanPer];
  int64_t v = 0;
  for (int k = 0; k < kScanPer; ++k) {
    c[k] = base + k < n ? counts[base + k] : 0;
    v += c[k];
  }
  int64_t run = block_incl_scan(v, sh) - v + tiles[blockIdx.x];
  for (int k = 0; k < kScanPer; ++k) {
    run += c[k];
    if (base + k < n) offsets[base + k + 1] = run;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) offsets[0] = 0;
}

hipError_t scan_counts(const int32_t *counts, int64_t *offsets, int64_t n, int64_t *tiles, hipStream_t st) {
  if (n <= 0) {
    launch_zero_u64(reinterpret_cast<unsigned long long *>(offsets), 1, st);
    return hipGetLastError();
  }
  const int64_t nt = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(scan_tile_sums, dim3((unsigned)nt), dim3(kScanThreads), 0, st, counts, n, tiles);
  hipLaunchKernelGGL(scan_tiles, dim3(1), dim3(kScanThreads), 0, st, tiles, nt);
  hipLaunchKernelGGL(scan_apply, dim3((unsigned)nt), dim3(kScanThreads), 0, st, counts, n, tiles, offsets);
  return hipGetLastError();
}

}  // namespace hfx

namespace hfx {

// ------------------------------------------------------- k-space assembly
// H(k)_{mu nu} = scale * sum_G K^G_{mu nu} exp(i k . (T_G + r_nu - r_mu)) for
// every k-point, dense complex (re, im interleaved) [nk][nbf][nbf].  One
// thread per (k, shell pair (I, J), element): it walks the pattern blocks
// (I, J, G) of the pair, which are contiguous, so no two threads write one
// entry.  Entries of shell pairs outside the pattern are zeroed by the
// caller.
__global__ __launch_bounds__(64) void kspace_kernel(DevSys s, const int4 *__restrict__ pairs, int npairs,
                                                    const int32_t *__restrict__ blk_img,
                                                    const int64_t *__restrict__ blk_off,
                                                    const int32_t *__restrict__ func_off, int sph,
                                                    const double *__restrict__ K, const double *__restrict__ kpts,
                                                    int nk, int64_t nbf, double scale, double *__restrict__ H) {
  const int p = blockIdx.x;
  const int k = blockIdx.y;
  if (p >= npairs || k >= nk) return;
  const int4 pr = pairs[p];  // I, J, first block, block count
  const int I = pr.x, J = pr.y;
  const int ni = nfunc_dev(s.sh_l[I], sph), nj = nfunc_dev(s.sh_l[J], sph);
  const int e = threadIdx.x;
  if (e >= ni * nj) return;
  const double kx = kpts[3 * k], ky = kpts[3 * k + 1], kz = kpts[3 * k + 2];
  const double dx = s.sh_xyz[3 * J] - s.sh_xyz[3 * I], dy = s.sh_xyz[3 * J + 1] - s.sh_xyz[3 * I + 1],
               dz = s.sh_xyz[3 * J + 2] - s.sh_xyz[3 * I + 2];
  double re = 0.0, im = 0.0;
  for (int b = pr.z; b < pr.z + pr.w; ++b) {
    int n1, n2, n3;
    unpack_img8(blk_img[b], n1, n2, n3);
    const double tx = n1 * s.lat[0] + n2 * s.lat[3] + n3 * s.lat[6] + dx;
    const double ty = n1 * s.lat[1] + n2 * s.lat[4] + n3 * s.lat[7] + dy;
    const double tz = n1 * s.lat[2] + n2 * s.lat[5] + n3 * s.lat[8] + dz;
    double sn, cs;
    sincos(kx * tx + ky * ty + kz * tz, &sn, &cs);
    const double v = K[blk_off[b] + e];
    re = fma(v, cs, re);
    im = fma(v, sn, im);
  }
  const int m = e / nj, n = e - m * nj;
  const int64_t row = func_off[I] + m, col = func_off[J] + n;
  double *h = H + 2 * (((int64_t)k * nbf + row) * nbf + col);
  h[0] = scale * re;
  h[1] = scale * im;
}

void launch_kspace(const DevSys &s, const int4 *pairs, int npairs, const int32_t *blk_img, const int64_t *blk_off,
                   const int32_t *func_off, int sph, const double *K, const double *kpts, int nk, int64_t nbf,
                   double scale, double *H, hipStream_t st) {
  launch_zero(H, 2 * (int64_t)nk * nbf * nbf, st);
  if (npairs <= 0 || nk <= 0) return;
  hipLaunchKernelGGL(kspace_kernel, dim3((unsigned)npairs, (unsigned)nk), dim3(64), 0, st, s, pairs, npairs, blk_img,
                     blk_off, func_off, sph, K, kpts, nk, nbf, scale, H);
}

}  // namespace hfx
