// Pieces shared by the one-wave-per-quartet ERI kernels (the cooperative LDS
// kernel and the lane-per-component kernel): staging of primitive-quartet
// prefactors, the HGP horizontal transfer of the contracted [e0|f0] held in
// LDS, and the four digest contributions into K.
#pragma once
#include "coop.hpp"
#include "os_hgp.hpp"

namespace hfx {

__device__ __forceinline__ double bcast(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// an empty asm that "modifies" x: the value is no longer loop-invariant to
// the optimiser
__device__ __forceinline__ void opaque(uint32_t &x) { asm volatile("" : "+v"(x)); }

__device__ __forceinline__ double sel3(int d, double x, double y, double z) { return d == 0 ? x : (d == 1 ? y : z); }
__device__ __forceinline__ double lds(const char *base, uint32_t byte_off) {
  return *reinterpret_cast<const double *>(base + byte_off);
}

// Primitive-quartet prefactors are computed a batch at a time (one lane each)
// and staged in LDS, kCoopStage doubles per primitive quartet:
//   [0, L]   ladder G_m times the prefactor (Boys or the erfc difference)
//   9..11    P - A        12..14  W - P
//   15..17   Q - C        18..20  W - Q
//   21 1/(2 zeta)  22 rho/zeta  23 1/(2 eta)  24 rho/eta  25 1/(2 (zeta + eta))
//   26 1.0  27 0.0 (coefficients of an identity step)
// The row stride is odd (29 doubles): rows written by consecutive lanes, and
// the rows different lane groups read at once, then fall in different LDS
// banks (an even stride of 28 left 2- to 16-way bank conflicts; measured 4%
// faster on the six-group lane kernels).
constexpr int kCoopBatch = 16;  // batch of the cooperative kernel
constexpr int kCoopStage = 29;
// LDS ints for the prefix sums of a ragged primitive-quartet set (<= 64 + 1)
constexpr int kPfxInts = kMaxPrim * kMaxPrim + 2;

// The primitive quartets of a contracted quartet that pass the bound
// threshold thr (0: all): bra primitive pair ib pairs with the first cnt(ib)
// ket primitive pairs (records sorted by bound).  Lane ib counts its ket
// pairs by bisection; pfx (nb + 1 ints, LDS) gets the exclusive prefix sums.
// Returns the number of primitive quartets (same in every lane).
__device__ __forceinline__ int prim_prefix(int *pfx, const double *__restrict__ ppb, int nb,
                                           const double *__restrict__ ppk, int nk, double thr, int lane) {
  int c = 0;
  if (lane < nb) {
    const double bthr = thr / ppb[(int64_t)lane * kPP + 9];
    int lo = 0, hi = nk;  // first ket pair below bthr
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (ppk[(int64_t)mid * kPP + 9] < bthr)
        hi = mid;
      else
        lo = mid + 1;
    }
    c = lo;
  }
  int x = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane < nb) pfx[lane + 1] = x;
  if (lane == 0) pfx[0] = 0;
  return __shfl(x, 63, 64);
}

// lanes 0 .. nbatch-1 stage primitive quartets t0 .. t0+nbatch-1 (those < n)
// of the set described by pfx
template <int L, int OP>
__device__ __forceinline__ void stage_prims(double *stage, int lane, int nbatch, int t0, int n, const int *pfx,
                                            int nb, const double *__restrict__ ppb, const double *__restrict__ ppk,
                                            double gx, double gy, double gz, const DevSys &s) {
  const int t = t0 + lane;
  if (lane < nbatch && t < n) {
    int lo = 0, hi = nb;  // last ib with pfx[ib] <= t
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pfx[mid] <= t)
        lo = mid;
      else
        hi = mid;
    }
    const int ib = lo, ik = t - pfx[lo];
    const double *b = ppb + (int64_t)ib * kPP;
    const double *k = ppk + (int64_t)ik * kPP;
    const double zeta = b[0], eta = k[0];
    const double rze = rsqrt_nr(zeta + eta);
    const double ize = rze * rze;
    const double rho = zeta * eta * ize;
    const double PQx = b[1] - (k[1] + gx), PQy = b[2] - (k[2] + gy), PQz = b[3] - (k[3] + gz);
    const double T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
    // 2 pi^(5/2) / (zeta eta sqrt(zeta + eta)) times the pair factors
    const double pref = b[7] * k[7] * rze;
    double G[L + 1];
    ladder<L, OP>(T, rho, s.omega2, pref, s.boys, G);
    const double fe = eta * ize, fz = zeta * ize;
    double *st = stage + lane * kCoopStage;
#pragma unroll
    for (int m = 0; m <= L; ++m) st[m] = G[m];
    st[9] = b[4]; st[10] = b[5]; st[11] = b[6];
    st[12] = -fe * PQx; st[13] = -fe * PQy; st[14] = -fe * PQz;
    st[15] = k[4]; st[16] = k[5]; st[17] = k[6];
    st[18] = fz * PQx; st[19] = fz * PQy; st[20] = fz * PQz;
    // rho/zeta = eta/(zeta+eta), rho/eta = zeta/(zeta+eta)
    st[21] = b[8]; st[22] = fe; st[23] = k[8]; st[24] = fz; st[25] = 0.5 * ize;
    st[26] = 1.0; st[27] = 0.0;
  }
}

// HRR of the contracted [e0|f0] (W[0, NE*NF), e-major) to (ab|cd) at
// W + cd.out_base, by the host-generated op list of the class.
template <int CB, int CK>
__device__ __forceinline__ void hrr_w(double *W, const CoopDev &cd, const DevSys &s, int bra, int ket, int lane) {
  const double *bg = s.pr_geom + (int64_t)bra * 8;
  const double *kg = s.pr_geom + (int64_t)ket * 8;
  const double ABx = bg[0], ABy = bg[1], ABz = bg[2], CDx = kg[0], CDy = kg[1], CDz = kg[2];
  for (int lv = cd.n_vrr_levels; lv < cd.n_vrr_levels + cd.n_hrr_levels; ++lv) {
    const int4 L4 = cd.levels[lv];
    const bool braside = (L4.z == kOpHrrBra);
    for (int it = lane; it < L4.y; it += 64) {
      const uint4 op = cd.ops[L4.x + it];
      const int o = op.x & 0xFFFF, a = op.x >> 16, b = op.y & 0xFFFF, dir = op.w & 3;
      const double f = braside ? sel3(dir, ABx, ABy, ABz) : sel3(dir, CDx, CDy, CDz);
      W[o] = W[a] + f * W[b];
    }
    __syncthreads();
  }
}

// Schwarz factor of bra pair (ab|ab): Q = sqrt(max |(ab|ab)|)
template <int CB>
__device__ __forceinline__ void schwarz_from_w(double *W, const CoopDev &cd, const DevSys &s, int bra, int lane) {
  hrr_w<CB, CB>(W, cd, s, bra, bra, lane);
  const double *v = W + cd.out_base;
  constexpr int NA = ncart(class_la(CB)), NB = ncart(class_lb(CB));
  double m = 0.0;
  for (int o = lane; o < NA * NB; o += 64) {
    const int a = o / NB, b = o - a * NB;
    m = fmax(m, fabs(v[((a * NB + b) * NA + a) * NB + b]));
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) m = fmax(m, __shfl_xor(m, d));
  if (lane == 0) s.pr_Q[bra] = sqrt(m);
}

// The four row-first digest contributions of one unique quartet (ab|cd) at v
// (row-major a, b, c, d) into K4, lanes over the output elements of each.
template <int CB, int CK>
__device__ __forceinline__ void digest_w(const double *v, const DevSys &s, int4 bi, int4 ki, int bra, int ket, int g1,
                                         int g2, int g3, const QuartetBlocks &qb, int lane) {
  constexpr int NA = ncart(class_la(CB)), NB = ncart(class_lb(CB)), NC = ncart(class_la(CK)),
                ND = ncart(class_lb(CK));
  const int bAC = qb.AC, bAD = qb.AD, bBC = qb.BC, bBD = qb.BD;
  double w = 1.0;
  if (bi.w & 1) w *= 0.5;
  if (ki.w & 1) w *= 0.5;
  if (bra == ket && g1 == 0 && g2 == 0 && g3 == 0) w *= 0.5;
  // a collinear-spin build digests the same integrals once per spin density
  for (int sp = 0; sp < s.nspin; ++sp) {
  const double *__restrict__ Dc = s.Dc + sp * s.spin_stride;
  double *__restrict__ K4 = s.K4 + sp * s.spin_stride;
  if (bAC >= 0 && bBD >= 0 && lane < NA * NC) {
    const double *D = Dc + s.blk_coff[bBD];
    const int a = lane / NC, c = lane - a * NC;
    double sum = 0.0;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int d = 0; d < ND; ++d) sum = fma(v[((a * NB + b) * NC + c) * ND + d], D[b * ND + d], sum);
    unsafeAtomicAdd(K4 + s.blk_coff[bAC] + lane, w * sum);
  }
  if (bBC >= 0 && bAD >= 0 && lane < NB * NC) {
    const double *D = Dc + s.blk_coff[bAD];
    const int b = lane / NC, c = lane - b * NC;
    double sum = 0.0;
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int d = 0; d < ND; ++d) sum = fma(v[((a * NB + b) * NC + c) * ND + d], D[a * ND + d], sum);
    unsafeAtomicAdd(K4 + s.blk_coff[bBC] + lane, w * sum);
  }
  if (bAD >= 0 && bBC >= 0 && lane < NA * ND) {
    const double *D = Dc + s.blk_coff[bBC];
    const int a = lane / ND, d = lane - a * ND;
    double sum = 0.0;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int c = 0; c < NC; ++c) sum = fma(v[((a * NB + b) * NC + c) * ND + d], D[b * NC + c], sum);
    unsafeAtomicAdd(K4 + s.blk_coff[bAD] + lane, w * sum);
  }
  if (bBD >= 0 && bAC >= 0 && lane < NB * ND) {
    const double *D = Dc + s.blk_coff[bAC];
    const int b = lane / ND, d = lane - b * ND;
    double sum = 0.0;
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int c = 0; c < NC; ++c) sum = fma(v[((a * NB + b) * NC + c) * ND + d], D[a * NC + c], sum);
    unsafeAtomicAdd(K4 + s.blk_coff[bBD] + lane, w * sum);
  }
  }
}

}  // namespace hfx
