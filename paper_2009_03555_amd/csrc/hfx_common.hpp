// Shared definitions of the MI355X exchange builder: device system view,
// compile-time Cartesian index algebra, quartet classes, packing.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hfx {

constexpr int kMaxL = 2;
constexpr int kMaxLT = 4 * kMaxL;     // highest Boys order of a quartet
constexpr int kMaxPrim = 8;
constexpr int kNPairClass = 6;        // ss ps pp ds dp dd (bra la >= lb)
constexpr int kNQuartetClass = 21;    // (cb, ck) with cb >= ck

// Boys table: F_m(T_i), T_i = i / 16, i = 0..640 (T < 40), m = 0..15, and
// exp(-T_i) in column 16.
constexpr int kBoysRows = 641;
constexpr int kBoysCols = 17;
constexpr double kBoysStep = 1.0 / 16.0;
constexpr double kBoysTmax = 40.0;

// ---------------------------------------------------------------- indexing
__host__ __device__ constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }
// number of Cartesian components of all levels below l
__host__ __device__ constexpr int noff(int l) { return l * (l + 1) * (l + 2) / 6; }

struct C3 {
  int x, y, z;
};
// component c of level l, order: x power descending, then y descending
__host__ __device__ constexpr C3 cart_of(int l, int c) {
  int a = 0;
  while ((a + 1) * (a + 2) / 2 <= c) ++a;  // a = l - x
  int z = c - a * (a + 1) / 2;
  return C3{l - a, a - z, z};
}
__host__ __device__ constexpr int cidx(C3 v) {
  int a = v.y + v.z;
  return a * (a + 1) / 2 + v.z;
}
__host__ __device__ constexpr int pw(C3 v, int i) { return i == 0 ? v.x : (i == 1 ? v.y : v.z); }
__host__ __device__ constexpr int dir_of(C3 v) { return v.x > 0 ? 0 : (v.y > 0 ? 1 : 2); }
__host__ __device__ constexpr C3 sub1(C3 v, int i) {
  return C3{v.x - (i == 0), v.y - (i == 1), v.z - (i == 2)};
}
__host__ __device__ constexpr C3 add1(C3 v, int i) {
  return C3{v.x + (i == 0), v.y + (i == 1), v.z + (i == 2)};
}
__host__ __device__ constexpr int cmax(int a, int b) { return a > b ? a : b; }

// pair classes: index -> (la, lb)
__host__ __device__ constexpr int class_la(int c) { return c == 0 ? 0 : (c <= 2 ? 1 : 2); }
__host__ __device__ constexpr int class_lb(int c) { return c == 0 ? 0 : (c == 1 ? 0 : (c == 2 ? 1 : c - 3)); }
__host__ __device__ constexpr int pair_class(int la, int lb) {
  return la == 0 ? 0 : (la == 1 ? 1 + lb : 3 + lb);
}
__host__ __device__ constexpr int region_of(int cb, int ck) { return cb * (cb + 1) / 2 + ck; }

// compile-time loop
template <int N>
struct IC {
  static constexpr int value = N;
};
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F &&f) {
  if constexpr (B < E) {
    f(IC<B>{});
    sfor<B + 1, E>(static_cast<F &&>(f));
  }
}

// --------------------------------------------------------------- packing
// image triple in a 5-bit-per-component field (components -16..15)
__host__ __device__ inline uint32_t pack_img5(int a, int b, int c) {
  return (uint32_t)(a + 16) | ((uint32_t)(b + 16) << 5) | ((uint32_t)(c + 16) << 10);
}
__host__ __device__ inline void unpack_img5(uint32_t p, int &a, int &b, int &c) {
  a = (int)(p & 31u) - 16;
  b = (int)((p >> 5) & 31u) - 16;
  c = (int)((p >> 10) & 31u) - 16;
}
// pair image triple, 8 bits per component
__host__ __device__ inline int32_t pack_img8(int a, int b, int c) {
  return (int32_t)((uint32_t)(a + 128) | ((uint32_t)(b + 128) << 8) | ((uint32_t)(c + 128) << 16));
}
__host__ __device__ inline void unpack_img8(int32_t p, int &a, int &b, int &c) {
  a = (int)(p & 255) - 128;
  b = (int)((p >> 8) & 255) - 128;
  c = (int)((p >> 16) & 255) - 128;
}
// quartet: bra pair (24 bits) | ket pair (24 bits) | ket translation (15 bits)
constexpr uint32_t kPairBits = 24;
constexpr uint32_t kMaxPairs = 1u << kPairBits;
__host__ __device__ inline uint64_t pack_quartet(uint32_t bra, uint32_t ket, uint32_t g) {
  return (uint64_t)bra | ((uint64_t)ket << 24) | ((uint64_t)g << 48);
}

// ------------------------------------------------------ device system view
// Primitive pair record (10 doubles): zeta, P(3), P-A(3),
// sqrt(2 pi^(5/2)) K / zeta with K = c_a c_b exp(-mu |AB|^2), 1/(2 zeta), and
// B, an upper bound of sqrt(|[p|p]|) over the pair's Cartesian components.
// The product of two such K/zeta factors times 1/sqrt(zeta + eta) is the
// primitive quartet's prefactor, so a quartet needs one division.  A pair's
// records are sorted by B, largest first.
constexpr int kPP = 10;
// A primitive quartet is skipped when B_bra B_ket P_scr < kPrimQuartetDrop:
// every integral it adds is below B_bra B_ket (Cauchy-Schwarz), so each of the
// at most 36 terms it adds to a K element is below 36 times this.  Measured
// on the 64-atom diamond cell against 1e-16: 1e-14 evaluates 14% fewer
// primitive quartets, builds 10% faster and moves K by at most 8.9e-12
// (|K| <= 2.3); 1e-13 moved it by 1.03e-10, past the 1e-10 bar.
constexpr double kPrimQuartetDrop = 1e-14;
constexpr double kSqrt2Pi52 = 5.914967172795612;  // sqrt(2 pi^(5/2))

struct DevSys {
  // shells
  const double *sh_xyz;   // [nsh*3]
  const int32_t *sh_l;    // [nsh]
  int32_t nsh;
  // unique pairs (evaluation orientation la >= lb)
  const int4 *pr_info;    // (A, B, packed image of B, flags bit0: A == B^n)
  const double *pr_geom;  // [np*8]: AB(3), midpoint M(3), radius r, unused
  const int2 *pr_pp;      // (offset into pp, number of significant prim pairs)
  const int32_t *pr_npp;  // all prim pairs (Schwarz uses all)
  double *pr_Q;           // Schwarz factor per unique pair
  int32_t npairs;
  const double *pp;       // [npp*kPP]
  // pattern / lookup
  const int32_t *lut;     // [(I*nsh + J)*nimg + img] -> block or -1
  int32_t imgR[3];
  int32_t nimg;
  const int64_t *blk_coff; // Cartesian value offset per block
  double *pmax;           // per block
  unsigned long long *pmax_global;  // bit pattern of max P (non-negative double)
  // lattice
  int32_t periodic;
  double lat[9];          // rows a1, a2, a3
  double rec[9];          // rows b1, b2, b3 with b_i . a_j = delta_ij
  double recn[3];         // |b_i|
  double cutoff;
  // operator
  int32_t op;             // 0 Coulomb, 1 erfc
  double omega2;
  double tau;
  // mixed precision, per class region: quartets with Q_IJ*Q_KL below this
  // go to the FP32 list (0: the class stays on the FP64 list)
  double fp32_cut[kNQuartetClass];
  const double *boys;     // kBoysRows x kBoysCols
  // per-build state of this plan
  const double *Dc;       // Cartesian density blocks (spin s at Dc + s * spin_stride)
  double *K4;             // Cartesian K accumulator (row-first contributions), same layout
  int32_t nspin;          // 1, or 2 for a collinear-spin build (both spins share every integral)
  int64_t spin_stride;    // Cartesian values per spin
  int32_t class_start[kNPairClass + 1];  // unique pairs of class c: [class_start[c], class_start[c+1])
};

// Plan of quartet qi in a fused class segment: seg[i] <= qi < seg[i+1]
// (seg has nsys + 1 entries; empty plans have seg[i] == seg[i+1]).
__device__ __forceinline__ int plan_of(const int64_t *__restrict__ seg, int nsys, int64_t qi) {
  int lo = 0, hi = nsys;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (seg[mid] <= qi)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// plan_of for a thread whose quartet index only grows: the plan of its
// previous quartet (hint) or the next one are checked first (one or two
// cached loads instead of a binary search over the bounds)
__device__ __forceinline__ int plan_of_hint(const int64_t *__restrict__ seg, int nsys, int64_t qi, int hint) {
  if (qi < seg[hint + 1]) return hint;
  if (hint + 2 <= nsys && qi < seg[hint + 2]) return hint + 1;
  return plan_of(seg, nsys, qi);
}

__device__ __forceinline__ int img_index(const DevSys &s, int a, int b, int c);
__device__ __forceinline__ int lookup(const DevSys &s, int I, int J, int a, int b, int c);

// The four digest blocks of quartet (A^0 B^nB | C^G D^(G+nD)): AC, AD, BC,
// BD (-1 if outside the pattern), and P_scr = the largest of their P_max.
struct QuartetBlocks {
  int AC, AD, BC, BD;
  double pscr;
};
__device__ __forceinline__ QuartetBlocks quartet_blocks(const DevSys &s, int4 bi, int4 ki, int g1, int g2, int g3) {
  int nB1, nB2, nB3, nD1, nD2, nD3;
  unpack_img8(bi.z, nB1, nB2, nB3);
  unpack_img8(ki.z, nD1, nD2, nD3);
  QuartetBlocks qb;
  qb.AC = lookup(s, bi.x, ki.x, g1, g2, g3);
  qb.AD = lookup(s, bi.x, ki.y, g1 + nD1, g2 + nD2, g3 + nD3);
  qb.BC = lookup(s, bi.y, ki.x, g1 - nB1, g2 - nB2, g3 - nB3);
  qb.BD = lookup(s, bi.y, ki.y, g1 + nD1 - nB1, g2 + nD2 - nB2, g3 + nD3 - nB3);
  double p = 0.0;
  if (qb.AC >= 0) p = fmax(p, s.pmax[qb.AC]);
  if (qb.AD >= 0) p = fmax(p, s.pmax[qb.AD]);
  if (qb.BC >= 0) p = fmax(p, s.pmax[qb.BC]);
  if (qb.BD >= 0) p = fmax(p, s.pmax[qb.BD]);
  qb.pscr = p;
  return qb;
}
// bound below which a primitive quartet of this quartet is skipped
__device__ __forceinline__ double prim_threshold(double pscr) {
  return pscr > 0.0 ? kPrimQuartetDrop / pscr : 1e300;
}

__device__ __forceinline__ int img_index(const DevSys &s, int a, int b, int c) {
  if (a < -s.imgR[0] || a > s.imgR[0] || b < -s.imgR[1] || b > s.imgR[1] || c < -s.imgR[2] ||
      c > s.imgR[2])
    return -1;
  return ((a + s.imgR[0]) * (2 * s.imgR[1] + 1) + (b + s.imgR[1])) * (2 * s.imgR[2] + 1) + (c + s.imgR[2]);
}

__device__ __forceinline__ int lookup(const DevSys &s, int I, int J, int a, int b, int c) {
  int k = img_index(s, a, b, c);
  if (k < 0) return -1;
  return s.lut[((int64_t)I * s.nsh + J) * s.nimg + k];
}

}  // namespace hfx
