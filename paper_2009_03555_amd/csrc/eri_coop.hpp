// Wave-cooperative ERI + digest kernel for high angular-momentum classes
// (see coop.hpp).  Per class, the level structure of the VRR is known at
// compile time, so each lane keeps its share of the VRR op list in registers
// for the whole launch and every level is pure LDS traffic plus FMAs.
#pragma once
#include "coop.hpp"
#include "launchers.hpp"
#include "os_hgp.hpp"

namespace hfx {

template <int CB, int CK, int GL = 64>
struct CoopShape {
  static constexpr int LA = class_la(CB), LB = class_lb(CB), LC = class_la(CK), LD = class_lb(CK);
  static constexpr int EB = LA + LB, FK = LC + LD, L = EB + FK;
  static constexpr int NLV = EB + FK;  // VRR levels: e = 1..EB, then f = 1..FK
  __host__ __device__ static constexpr int count(int lv) {
    if (lv < EB) return ncart(lv + 1) * (L - lv);
    const int f = lv - EB + 1;
    const int elo = cmax(0, LA - (FK - f));
    return ncart(f) * (noff(EB + 1) - noff(elo)) * (FK - f + 1);
  }
  __host__ __device__ static constexpr int rounds(int lv) { return (count(lv) + GL - 1) / GL; }
  __host__ __device__ static constexpr int round_base(int lv) {
    int s = 0;
    for (int i = 0; i < lv; ++i) s += rounds(i);
    return s;
  }
  __host__ __device__ static constexpr int op_base(int lv) {  // padded layout
    int s = 0;
    for (int i = 0; i < lv; ++i) s += rounds(i) * GL;
    return s;
  }
  static constexpr int NR = round_base(NLV);
  static constexpr int NACC = (noff(EB + 1) - noff(LA)) * (noff(FK + 1) - noff(LC));
  static constexpr int SLOTS = (NACC + 63) / 64;
};

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

// P primitive quartets of one contracted quartet are evaluated side by side:
// lane group g (GL = 64 / P lanes) runs the VRR of its primitive quartet in its
// own LDS workspace; prefactors are computed 16 at a time and staged in LDS.
constexpr int kCoopBatch = 16;
constexpr int kCoopStage = 26;  // doubles staged per primitive quartet: ladder (<= 9) + 17 factors

// MODE 0: ERI + digest over a quartet list.  MODE 1: Schwarz factors of the
// pairs p0 .. p0+nq-1 of class CB (= CK): (ab|ab) over all primitive pairs,
// Q_p = sqrt(max |(ab|ab)|) written to s.pr_Q.
template <int CB, int CK, int OP, int P, int MODE>
__global__ __launch_bounds__(64) void eri_coop_kernel(const DevSys *__restrict__ sys, int nsys,
                                                      const int64_t *__restrict__ seg, CoopDev cd,
                                                      const uint64_t *__restrict__ list,
                                                      unsigned long long *__restrict__ nprim, int p0,
                                                      int64_t npairs) {
  constexpr int GL = 64 / P;
  using SH = CoopShape<CB, CK, GL>;
  using SH64 = CoopShape<CB, CK, 64>;
  constexpr int L = SH::L;
  extern __shared__ double W[];
  char *Wb = reinterpret_cast<char *>(W);
  const int lane = threadIdx.x;
  const int grp = lane / GL, gl = lane - grp * GL;
  const uint32_t wbase = (uint32_t)(grp * (cd.nw + 1) * 8);
  const int nws = cd.nw + 1;       // workspace doubles incl. the dummy slot
  double *stage = W + P * nws;     // kCoopBatch x kCoopStage
  // this lane's VRR ops for the whole launch
  uint32_t opA[SH::NR], opB[SH::NR];
  sfor<0, SH::NLV>([&](auto lv_) {
    constexpr int lv = decltype(lv_)::value;
    sfor<0, SH::rounds(lv)>([&](auto r_) {
      constexpr int r = decltype(r_)::value;
      constexpr int slot = SH::round_base(lv) + r;
      const uint4 o = cd.vops[SH::op_base(lv) + gl + GL * r];
      opA[slot] = o.x;
      opB[slot] = o.y;
    });
  });
  uint32_t accoff[SH64::SLOTS];
#pragma unroll
  for (int k = 0; k < SH64::SLOTS; ++k) {
    const int tt = k * 64 + lane;
    accoff[k] = tt < SH64::NACC ? 8u * cd.acc_off[tt] : 0u;
  }
  unsigned long long prims = 0;
  const int64_t q0 = MODE == 0 ? seg[0] : 0, q1 = MODE == 0 ? seg[nsys] : npairs;
  for (int64_t qi = q0 + blockIdx.x; qi < q1; qi += gridDim.x) {
    const DevSys &s = sys[(MODE == 0 && nsys > 1) ? plan_of(seg, nsys, qi) : 0];
    const double *__restrict__ Dc = s.Dc;
    double *__restrict__ K4 = s.K4;
    int bra, ket, g1 = 0, g2 = 0, g3 = 0;
    if constexpr (MODE == 0) {
      const uint64_t q = list[qi];
      bra = (int)(q & 0xFFFFFFull);
      ket = (int)((q >> 24) & 0xFFFFFFull);
      unpack_img5((uint32_t)(q >> 48), g1, g2, g3);
    } else {
      bra = ket = p0 + (int)qi;
    }
    const int4 bi = s.pr_info[bra], ki = s.pr_info[ket];
    int2 bpp = s.pr_pp[bra], kpp = s.pr_pp[ket];
    if constexpr (MODE == 1) {
      bpp.y = s.pr_npp[bra];
      kpp.y = bpp.y;
    }
    double gx = 0.0, gy = 0.0, gz = 0.0;
    if (s.periodic) {
      gx = g1 * s.lat[0] + g2 * s.lat[3] + g3 * s.lat[6];
      gy = g1 * s.lat[1] + g2 * s.lat[4] + g3 * s.lat[7];
      gz = g1 * s.lat[2] + g2 * s.lat[5] + g3 * s.lat[8];
    }
    const double *ppb = s.pp + (int64_t)bpp.x * kPP;
    const double *ppk = s.pp + (int64_t)kpp.x * kPP;
    const int nk = kpp.y;
    const int n = bpp.y * nk;
    prims += (unsigned long long)n;
    double acc[SH64::SLOTS];
#pragma unroll
    for (int k = 0; k < SH64::SLOTS; ++k) acc[k] = 0.0;

    for (int t0 = 0; t0 < n; t0 += kCoopBatch) {
      // stage prefactors of up to kCoopBatch primitive quartets
      const int t = t0 + lane;
      if (lane < kCoopBatch && t < n) {
        const int ib = t / nk, ik = t - ib * nk;
        const double *b = ppb + (int64_t)ib * kPP;
        const double *k = ppk + (int64_t)ik * kPP;
        const double zeta = b[0], eta = k[0];
        const double ze = zeta + eta, ize = 1.0 / ze;
        const double rho = zeta * eta * ize;
        const double PQx = b[1] - (k[1] + gx), PQy = b[2] - (k[2] + gy), PQz = b[3] - (k[3] + gz);
        const double T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
        const double pref = 34.986836655249725693 / (zeta * eta * sqrt(ze)) * b[7] * k[7];
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
        st[21] = 0.5 / zeta; st[22] = rho / zeta; st[23] = 0.5 / eta; st[24] = rho / eta; st[25] = 0.5 * ize;
      }
      __syncthreads();
      const int cnt = (n - t0) < kCoopBatch ? (n - t0) : kCoopBatch;
      for (int u0 = 0; u0 < cnt; u0 += P) {
        const int u = u0 + grp;
        const bool live = u < cnt;
        const double *st = stage + (live ? u : 0) * kCoopStage;
        // direction-dependent factors are read from the stage by address
        const uint32_t stb = (uint32_t)(reinterpret_cast<const char *>(st) - Wb);
        const double uo2z = st[21], urz = st[22], uo2e = st[23], ure = st[24], uo2ze = st[25];
        if (gl <= L) *reinterpret_cast<double *>(Wb + wbase + 8 * gl) = live ? st[gl] : 0.0;
        // the op words are loop-invariant per lane; keep the compiler from
        // hoisting per-round masks derived from them into (spilled) SGPRs
        sfor<0, SH::NR>([&](auto k_) {
          opaque(opA[decltype(k_)::value]);
          opaque(opB[decltype(k_)::value]);
        });
        __syncthreads();
        sfor<0, SH::NLV>([&](auto lv_) {
          constexpr int lv = decltype(lv_)::value;
          constexpr bool braside = lv < SH::EB;
          sfor<0, SH::rounds(lv)>([&](auto r_) {
            constexpr int r = decltype(r_)::value;
            constexpr int slot = SH::round_base(lv) + r;
            {
              // branch-free: absent terms have coefficient 0 and read slot 0
              const uint32_t A = opA[slot], B = opB[slot];
              const uint32_t o = wbase + (A & 0xFFF8u), a = wbase + ((A >> 16) & 0xFFF8u);
              const uint32_t c = wbase + (B & 0xFFF8u);
              const uint32_t cf = stb + ((B & 3u) << 3);
              const double nn = (double)((A >> 16) & 7u);
              double rr;
              if constexpr (braside) {
                // PA[dir] at stage 9 + dir, (W-P)[dir] at 12 + dir
                rr = lds(Wb, cf + 72) * lds(Wb, a) + lds(Wb, cf + 96) * lds(Wb, a + 8);
                rr += nn * uo2z * (lds(Wb, c) - urz * lds(Wb, c + 8));
              } else {
                // QC[dir] at stage 15 + dir, (W-Q)[dir] at 18 + dir
                const double ne = (double)(A & 7u);
                rr = lds(Wb, cf + 120) * lds(Wb, a) + lds(Wb, cf + 144) * lds(Wb, a + 8);
                rr += nn * uo2e * (lds(Wb, c) - ure * lds(Wb, c + 8));
                rr += ne * uo2ze * lds(Wb, wbase + (B >> 16));
              }
              *reinterpret_cast<double *>(Wb + o) = rr;
            }
          });
          __syncthreads();
        });
        // targets of every live workspace
#pragma unroll
        for (int k = 0; k < SH64::SLOTS; ++k) {
          if (k + 1 < SH64::SLOTS || k * 64 + lane < SH64::NACC) {
#pragma unroll
            for (int g = 0; g < P; ++g)
              if (u0 + g < cnt) acc[k] += lds(Wb, (uint32_t)(g * nws * 8) + accoff[k]);
          }
        }
        __syncthreads();
      }
    }
    // contracted targets -> HRR (op list from memory: once per contracted quartet)
#pragma unroll
    for (int k = 0; k < SH64::SLOTS; ++k) {
      const int tt = k * 64 + lane;
      if (tt < SH64::NACC) W[tt] = acc[k];
    }
    __syncthreads();
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
    const double *v = W + cd.out_base;
    constexpr int NA = ncart(SH::LA), NB = ncart(SH::LB), NC = ncart(SH::LC), ND = ncart(SH::LD);
    if constexpr (MODE == 1) {
      double m = 0.0;
      for (int o = lane; o < NA * NB; o += 64) {
        const int a = o / NB, b = o - a * NB;
        m = fmax(m, fabs(v[((a * NB + b) * NA + a) * NB + b]));
      }
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) m = fmax(m, __shfl_xor(m, d));
      if (lane == 0) s.pr_Q[bra] = sqrt(m);
      __syncthreads();
      continue;
    }
    // digest: lanes over the output elements of each contribution
    int nB1, nB2, nB3, nD1, nD2, nD3;
    unpack_img8(bi.z, nB1, nB2, nB3);
    unpack_img8(ki.z, nD1, nD2, nD3);
    const int A = bi.x, B = bi.y, Cs = ki.x, Ds = ki.y;
    const int bAC = lookup(s, A, Cs, g1, g2, g3);
    const int bAD = lookup(s, A, Ds, g1 + nD1, g2 + nD2, g3 + nD3);
    const int bBC = lookup(s, B, Cs, g1 - nB1, g2 - nB2, g3 - nB3);
    const int bBD = lookup(s, B, Ds, g1 + nD1 - nB1, g2 + nD2 - nB2, g3 + nD3 - nB3);
    double w = 1.0;
    if (bi.w & 1) w *= 0.5;
    if (ki.w & 1) w *= 0.5;
    if (bra == ket && g1 == 0 && g2 == 0 && g3 == 0) w *= 0.5;
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
    __syncthreads();
  }
  if constexpr (MODE == 0)
    if (lane == 0 && prims) atomicAdd(nprim, prims);
}

// primitive quartets evaluated side by side per wave, by class size
template <int CB, int CK, int OP>
void launch_coop_t(const CoopDev &cd, const SegLaunch &L) {
  if (L.nq_hint == 0) return;
  constexpr int P = coop_parallel(CB, CK);
  const int64_t blocks = (L.nq_hint > 0 && L.nq_hint < 256 * 32) ? L.nq_hint : 256 * 32;
  const size_t lds = ((size_t)P * (cd.nw + 1) + (size_t)kCoopBatch * kCoopStage) * sizeof(double);
  hipLaunchKernelGGL((eri_coop_kernel<CB, CK, OP, P, 0>), dim3((unsigned)blocks), dim3(64), lds, L.stream, L.sys,
                     L.nsys, L.seg, cd, L.list, L.nprim, 0, (int64_t)0);
}

// sys1: device descriptor of the one plan whose pairs p0 .. p1-1 are processed
template <int CB, int OP>
void launch_coop_schwarz_t(const DevSys *sys1, const CoopDev &cd, int p0, int p1, hipStream_t st) {
  if (p1 <= p0) return;
  constexpr int P = coop_parallel(CB, CB);
  const int64_t n = p1 - p0;
  const int64_t blocks = n < 256 * 32 ? n : 256 * 32;
  const size_t lds = ((size_t)P * (cd.nw + 1) + (size_t)kCoopBatch * kCoopStage) * sizeof(double);
  hipLaunchKernelGGL((eri_coop_kernel<CB, CB, OP, P, 1>), dim3((unsigned)blocks), dim3(64), lds, st, sys1, 1,
                     (const int64_t *)nullptr, cd, (const uint64_t *)nullptr, (unsigned long long *)nullptr, p0,
                     n);
}

}  // namespace hfx

#define HFX_COOP_SCHWARZ_UNIT(CB)                                                                    \
  namespace hfx {                                                                                    \
  void launch_schwarz_coop_c##CB(int op, const DevSys *sys1, const CoopDev &cd, int p0, int p1,     \
                                 hipStream_t st) {                                                   \
    if (op == 0)                                                                                     \
      launch_coop_schwarz_t<CB, 0>(sys1, cd, p0, p1, st);                                            \
    else                                                                                             \
      launch_coop_schwarz_t<CB, 1>(sys1, cd, p0, p1, st);                                            \
  }                                                                                                  \
  }

#define HFX_COOP_UNIT(CB, CK)                                                                        \
  namespace hfx {                                                                                    \
  void launch_eri_coop_r##CB##CK(int op, const CoopDev &cd, const SegLaunch &L) {                  \
    if (op == 0)                                                                                     \
      launch_coop_t<CB, CK, 0>(cd, L);                                                               \
    else                                                                                             \
      launch_coop_t<CB, CK, 1>(cd, L);                                                               \
  }                                                                                                  \
  }
