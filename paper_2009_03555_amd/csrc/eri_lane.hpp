// Lane-per-component ERI + digest kernel for high angular-momentum classes.
//
// The Obara-Saika VRR to [e0|f0] is split by electron.  One side (the "lane
// side", the pair class with the lower total angular momentum) is spread over
// the lanes of a group: lane s owns the Cartesian component s of that side's
// levels 0..LS.  The other side (the "grow side") is built last, entirely in
// that lane's registers, by the compile-time-unrolled recursion on the grow
// index: every operand of the grow-side step is lane-local except the
// electron-coupling term N_i(s)/(2(zeta+eta)) [s - 1_i, g]^(m+1), which one
// LDS read fetches from the lane owning s - 1_i.  A group needs
// noff(LS + 1) lanes; 64 / that many groups evaluate different primitive
// quartets of the same contracted quartet side by side.  Each lane sums its
// targets [s, g]^(0) over the primitive quartets in registers; the groups are
// combined by cross-lane reads once per contracted quartet, followed by the
// HGP HRR and the digest in LDS.
//
// Before the grow-side build, each lane needs [s, 0]^(m): it walks the chain
// of ancestors of s (the unique build path of the lane side's recursion)
// itself, which costs no more wave time than a shared level-by-level build.
#pragma once
#include "eri_wave.hpp"
#include "launchers.hpp"


namespace hfx {

template <int CB, int CK, bool KL>
struct LaneShape {
  static constexpr int LA = class_la(CB), LB = class_lb(CB), LC = class_la(CK), LD = class_lb(CK);
  static constexpr int EB = LA + LB, FK = LC + LD, L = EB + FK;
  static constexpr int LS = KL ? FK : EB;  // lane side: components of levels 0..LS
  static constexpr int SL = KL ? LC : LA;  // lowest lane-side level among the targets
  static constexpr int LG = KL ? EB : FK;  // grow side, built in registers
  static constexpr int GL = KL ? LA : LC;  // lowest grow-side level among the targets
  static constexpr int NS = noff(LS + 1);
  static constexpr int NGRP = 64 / NS;
  static constexpr int NGT = noff(LG + 1) - noff(GL);
  // read a whole level's coupling operands at once: measured faster where
  // the registers allow it (grow side up to L = 3, (dd|dd), which runs one
  // wave per SIMD either way, and every FP32 kernel)
  template <typename TV>
  static constexpr bool batch_reads() {
    return LG <= 3 || (CB == 5 && CK == 5) || sizeof(TV) == 4;
  }
  static constexpr int NE = noff(EB + 1) - noff(LA), NF = noff(FK + 1) - noff(LC);
  static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
  // primitive quartets staged per batch, a multiple of the group count:
  // about 32, or 60 for six groups with a grow side up to L = 3 and for the
  // FP64 (dp|dp) kernel (measured 8% and 5% faster there; elsewhere the
  // larger LDS footprint costs waves per CU, as it would for the FP32
  // (dp|dp) kernel, which runs three waves per SIMD)
  template <typename TV>
  static constexpr int nbatch() {
    return ((NGRP == 6 && LG <= 3) || (sizeof(TV) == 8 && CB == 4 && CK == 4)) ? 60
                                                                              : NGRP * ((32 + NGRP - 1) / NGRP);
  }
  // register slots V[lv][c][m], m = 0..LG-lv
  __host__ __device__ static constexpr int vw(int lv) { return LG - lv + 1; }
  __host__ __device__ static constexpr int vo(int lv, int c, int m) {
    int s = 0;
    for (int l = 0; l < lv; ++l) s += ncart(l) * vw(l);
    return s + c * vw(lv) + m;
  }
  static constexpr int NV = vo(LG + 1, 0, 0);
  // published values of one level: (c, m = 1..LG-lv) at c*(LG-lv) + m-1, for
  // each of the 64 lanes; two buffers alternate by level
  __host__ __device__ static constexpr int pbl() {
    int m = 1;
    for (int l = 0; l < LG; ++l) m = cmax(m, ncart(l) * (LG - l));
    return m;
  }
  // HRR ping-pong region: twice the largest HRR level (same as the op lists)
  __host__ __device__ static constexpr int hrr_r() {
    int r = NE * NF;
    for (int b = 1; b <= LB; ++b) r = cmax(r, (noff(EB - b + 1) - noff(LA)) * ncart(b) * NF);
    for (int d = 1; d <= LD; ++d) r = cmax(r, NA * NB * (noff(FK - d + 1) - noff(LC)) * ncart(d));
    return r;
  }
  // publish buffers during the primitive loop, the HRR region after it
  template <typename TV>
  __host__ __device__ static constexpr int work_doubles() {
    return cmax(2 * hrr_r(), (2 * pbl() * 64 * (int)sizeof(TV) + 7) / 8);
  }
  template <typename TV>
  __host__ __device__ static constexpr size_t lds_bytes() {
    return (size_t)(work_doubles<TV>() + nbatch<TV>() * kCoopStage) * sizeof(double) + kPfxInts * sizeof(int);
  }
};

// LDS ordering between the lanes of the one wave of a work-group: a wave's
// LDS operations complete in issue order, so a wavefront-scope fence (no
// wait) and a compiler barrier suffice
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The electron-coupling operands cross lanes through LDS: each level is
// published and read back (register shuffles measured slower)
// FP64: two waves per SIMD wanted, a register budget of 256 per lane; the
// (dd|dd) kernel needs more and runs one wave per SIMD.  FP32: three waves
// for (dp|dp), (dd|pp), (dd|ds) (measured 2-14% faster despite a few spilled
// registers); elsewhere three cost more than they gain, or the kernel gets
// there by itself
template <int CB, int CK, typename TV>
constexpr int lane_waves() {
  if constexpr (sizeof(TV) == 4) {
    if ((CB == 4 && CK == 4) || (CB == 5 && (CK == 2 || CK == 3))) return 3;
  }
  return (CB == 5 && CK == 5) ? 1 : 2;
}

template <int CB, int CK, int OP, bool KL, typename TV>
__global__ __attribute__((amdgpu_flat_work_group_size(64, 64), amdgpu_waves_per_eu(lane_waves<CB, CK, TV>())))
void eri_lane_kernel(const DevSys *__restrict__ sys, int nsys,
                                                      const int64_t *__restrict__ seg, CoopDev cd,
                                                      const uint64_t *__restrict__ list,
                                                      unsigned long long *__restrict__ nprim) {
  using SH = LaneShape<CB, CK, KL>;
  constexpr int L = SH::L, LS = SH::LS, LG = SH::LG, GL = SH::GL, NS = SH::NS, NGRP = SH::NGRP;
  constexpr int NGT = SH::NGT, NF = SH::NF, PBL = SH::pbl(), NBATCH = SH::template nbatch<TV>();
  // stage slots of the lane side and of the grow side
  constexpr int XS = KL ? 15 : 9, YS = KL ? 18 : 12, OS2 = KL ? 23 : 21, RS = KL ? 24 : 22;
  constexpr int XG = KL ? 9 : 15, YG = KL ? 12 : 18, OG2 = KL ? 21 : 23, RG = KL ? 22 : 24;
  extern __shared__ double W[];
  TV *pub = reinterpret_cast<TV *>(W);
  double *stage = W + SH::template work_doubles<TV>();
  int *pfx = reinterpret_cast<int *>(stage + NBATCH * kCoopStage);
  const int lane = threadIdx.x;
  // The published values of a level: row r, lane l at pub[r * 64 + l].
  // FP64 with twenty-lane groups: as two 32-bit planes (low words at
  // [r * 128 + l], high words 64 further), read by 32-bit accesses; 64-bit
  // reads of two groups' parents in one 16-lane pass hit the same banks
  // (measured 3% faster on (dd|dp), bank-conflict cycles near zero)
  constexpr bool kSplit = NS == 20 && sizeof(TV) == 8;
  uint32_t *pub32 = reinterpret_cast<uint32_t *>(W);
  auto pub_put = [&](int row, TV v) {
    if constexpr (kSplit) {
      const unsigned long long b = (unsigned long long)__double_as_longlong((double)v);
      pub32[row * 128 + lane] = (uint32_t)b;
      pub32[row * 128 + 64 + lane] = (uint32_t)(b >> 32);
    } else {
      pub[row * 64 + lane] = v;
    }
  };
  auto pub_get = [&](int row, int from) -> TV {
    if constexpr (kSplit) {
      const uint32_t lo = pub32[row * 128 + from], hi = pub32[row * 128 + 64 + from];
      return (TV)__longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    } else {
      return pub[row * 64 + from];
    }
  };
  const bool active = lane < NGRP * NS;
  const int grp = active ? lane / NS : 0;
  const int sidx = active ? lane - grp * NS : 0;
  int ns = 0;
  while (noff(ns + 1) <= sidx) ++ns;
  const C3 sc = cart_of(ns, sidx - noff(ns));
  // electron-coupling term: power s_i and the lane of s - 1_i.  Where the
  // term vanishes (s_i = 0) the lane reads its group's first lane instead of
  // its own, and idle lanes read the last group's first lane: the value is
  // multiplied by zero, and a read then touches only the parents of the
  // groups in each 16-lane pass, which fall in distinct LDS banks (own-lane
  // reads made 2-way bank conflicts; measured 3-5% faster without them)
  int src[3];
  TV npow[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int n = pw(sc, i);
    npow[i] = (TV)n;
    src[i] = !active ? (NGRP - 1) * NS : (n > 0 ? grp * NS + noff(ns - 1) + cidx(sub1(sc, i)) : grp * NS);
  }
  // ancestor chain of s, shifted so that every lane ends at step LS: lane
  // level j = k - (LS - ns) is built at step k; earlier steps are identities
  // (X = 1, Y = 0, no second term), which keep [0]^(m) with the m range every
  // step needs (m <= L - k for all lanes).  xo/yo: stage slots of X and Y,
  // cpw: the parent's power in the build direction.
  int xo[LS > 0 ? LS : 1], yo[LS > 0 ? LS : 1];
  TV cpw[LS > 0 ? LS : 1];
#pragma unroll
  for (int k = 1; k <= LS; ++k) {
    const int j = k - (LS - ns);
    C3 cur = sc;  // walk down to the ancestor at level j
#pragma unroll
    for (int t = 0; t < LS; ++t)
      if (t < ns - j) cur = sub1(cur, dir_of(cur));
    int d = 0, np = 0;
    if (j >= 1) {
      d = dir_of(cur);
      np = pw(sub1(cur, d), d);
    }
    xo[k - 1] = j >= 1 ? XS + d : 26;
    yo[k - 1] = j >= 1 ? YS + d : 27;
    cpw[k - 1] = (TV)np;
  }

  // lane-local part of grow component c of level lv, all m:
  // X_i [g]^(m) + Y_i [g]^(m+1) + N_i(g)/(2 zeta_g) ([g-1_i]^(m) - rho/zeta_g [g-1_i]^(m+1)),
  // g = t - 1_i the parent in the build direction i of t
  auto grow_local = [&]<int lv, int c>(TV *V, const TV *gX, const TV *gY, TV o2g, TV rg) {
    constexpr int MR = LG - lv;
    constexpr C3 t = cart_of(lv, c);
    constexpr int i = dir_of(t);
    constexpr C3 p = sub1(t, i);
    constexpr int np = pw(p, i);
    constexpr int pc = cidx(p);
    constexpr int ppc = np > 0 ? cidx(sub1(p, i)) : 0;
#pragma unroll
    for (int m = 0; m <= MR; ++m) {
      TV v = fma(gY[i], V[SH::vo(lv - 1, pc, m + 1)], gX[i] * V[SH::vo(lv - 1, pc, m)]);
      if constexpr (np > 0)
        v = fma((TV)np * o2g, fma(-rg, V[SH::vo(lv - 2, ppc, m + 1)], V[SH::vo(lv - 2, ppc, m)]), v);
      V[SH::vo(lv, c, m)] = v;
    }
  };
  unsigned long long prims = 0;
  const int64_t q0 = seg[0], q1 = seg[nsys];
  int pl = 0;  // plan of the previous quartet
  for (int64_t qi = q0 + blockIdx.x; qi < q1; qi += gridDim.x) {
    pl = nsys > 1 ? plan_of_hint(seg, nsys, qi, pl) : 0;
    const DevSys &s = sys[pl];
    const uint64_t q = list[qi];
    const int bra = (int)(q & 0xFFFFFFull), ket = (int)((q >> 24) & 0xFFFFFFull);
    int g1, g2, g3;
    unpack_img5((uint32_t)(q >> 48), g1, g2, g3);
    const int4 bi = s.pr_info[bra], ki = s.pr_info[ket];
    const int2 bpp = s.pr_pp[bra], kpp = s.pr_pp[ket];
    double gx = 0.0, gy = 0.0, gz = 0.0;
    if (s.periodic) {
      gx = g1 * s.lat[0] + g2 * s.lat[3] + g3 * s.lat[6];
      gy = g1 * s.lat[1] + g2 * s.lat[4] + g3 * s.lat[7];
      gz = g1 * s.lat[2] + g2 * s.lat[5] + g3 * s.lat[8];
    }
    const double *ppb = s.pp + (int64_t)bpp.x * kPP;
    const double *ppk = s.pp + (int64_t)kpp.x * kPP;
    // with a d-d grow side the digest looks its blocks up again, so that
    // nothing of this stays live through the primitive loop (registers)
    const QuartetBlocks qb = quartet_blocks(s, bi, ki, g1, g2, g3);
    const int n = prim_prefix(pfx, ppb, bpp.y, ppk, kpp.y, prim_threshold(qb.pscr), lane);
    prims += (unsigned long long)n;
    __syncthreads();
    TV acc[NGT];
#pragma unroll
    for (int k = 0; k < NGT; ++k) acc[k] = (TV)0;

    for (int t0 = 0; t0 < n; t0 += NBATCH) {
      stage_prims<L, OP>(stage, lane, NBATCH, t0, n, pfx, bpp.y, ppb, ppk, gx, gy, gz, s);
      __syncthreads();
      const int cnt = (n - t0) < NBATCH ? (n - t0) : NBATCH;
      for (int u0 = 0; u0 < cnt; u0 += NGRP) {
        const int u = u0 + grp;
        const bool live = u < cnt;
        const double *st = stage + (live ? u : 0) * kCoopStage;
        const TV o2s = (TV)st[OS2], rs = (TV)st[RS];
        const TV gX[3] = {(TV)st[XG], (TV)st[XG + 1], (TV)st[XG + 2]};
        const TV gY[3] = {(TV)st[YG], (TV)st[YG + 1], (TV)st[YG + 2]};
        const TV o2g = (TV)st[OG2], rg = (TV)st[RG];
        const TV o2ze = (TV)st[25];
        const TV xc[3] = {npow[0] * o2ze, npow[1] * o2ze, npow[2] * o2ze};

        // ---- lane side: [s, 0]^(m), m = 0..LG, along the ancestor chain
        TV cur[L + 1], prv[L + 1];
#pragma unroll
        for (int m = 0; m <= L; ++m) cur[m] = live ? (TV)st[m] : (TV)0;
#pragma unroll
        for (int m = 0; m <= L; ++m) prv[m] = (TV)0;
        sfor<1, LS + 1>([&](auto k_) {
          constexpr int k = decltype(k_)::value;
          constexpr int MK = L - k;
          const TV X = (TV)st[xo[k - 1]], Y = (TV)st[yo[k - 1]];
          const TV cn = cpw[k - 1] * o2s;
          TV nw[MK + 1];
#pragma unroll
          for (int m = 0; m <= MK; ++m) {
            TV v = fma(Y, cur[m + 1], X * cur[m]);
            if constexpr (k >= 2) v = fma(cn, fma(-rs, prv[m + 1], prv[m]), v);
            nw[m] = v;
          }
#pragma unroll
          for (int m = 0; m <= MK + 1; ++m) prv[m] = cur[m];
#pragma unroll
          for (int m = 0; m <= MK; ++m) cur[m] = nw[m];
        });

        // ---- grow side in registers, electron coupling through LDS
        TV V[SH::NV];
#pragma unroll
        for (int m = 0; m <= LG; ++m) V[SH::vo(0, 0, m)] = cur[m];
        if constexpr (GL == 0) acc[0] += V[0];
        if constexpr (LG > 0) {
#pragma unroll
          for (int m = 1; m <= LG; ++m) pub_put(m - 1, V[SH::vo(0, 0, m)]);
          wave_lds_sync();
        }
        sfor<1, LG + 1>([&](auto lv_) {
          constexpr int lv = decltype(lv_)::value;
          constexpr int MR = LG - lv;
          constexpr int rb = ((lv - 1) & 1) * PBL, wb = (lv & 1) * PBL;
          if constexpr (SH::template batch_reads<TV>()) {
            // every electron-coupling operand of the level first (one
            // wait), the lane-local terms while they arrive, then the
            // coupling terms
            TV RL[ncart(lv) * (MR + 1)];
            sfor<0, ncart(lv)>([&](auto c_) {
              constexpr int c = decltype(c_)::value;
              constexpr int i = dir_of(cart_of(lv, c));
              constexpr int pc = cidx(sub1(cart_of(lv, c), i));
#pragma unroll
              for (int m = 0; m <= MR; ++m) RL[c * (MR + 1) + m] = pub_get(rb + pc * (MR + 1) + m, src[i]);
            });
            sfor<0, ncart(lv)>([&](auto c_) {
              constexpr int c = decltype(c_)::value;
              grow_local.template operator()<lv, c>(V, gX, gY, o2g, rg);
            });
            sfor<0, ncart(lv)>([&](auto c_) {
              constexpr int c = decltype(c_)::value;
              constexpr int i = dir_of(cart_of(lv, c));
#pragma unroll
              for (int m = 0; m <= MR; ++m)
                V[SH::vo(lv, c, m)] = fma(xc[i], RL[c * (MR + 1) + m], V[SH::vo(lv, c, m)]);
              if constexpr (lv >= GL) acc[noff(lv) + c - noff(GL)] += V[SH::vo(lv, c, 0)];
            });
          } else {
            // component by component (register budget of the d-d grow side)
            sfor<0, ncart(lv)>([&](auto c_) {
              constexpr int c = decltype(c_)::value;
              constexpr int i = dir_of(cart_of(lv, c));
              constexpr int pc = cidx(sub1(cart_of(lv, c), i));
              TV R[MR + 1];
#pragma unroll
              for (int m = 0; m <= MR; ++m) R[m] = pub_get(rb + pc * (MR + 1) + m, src[i]);
              grow_local.template operator()<lv, c>(V, gX, gY, o2g, rg);
#pragma unroll
              for (int m = 0; m <= MR; ++m) V[SH::vo(lv, c, m)] = fma(xc[i], R[m], V[SH::vo(lv, c, m)]);
              if constexpr (lv >= GL) acc[noff(lv) + c - noff(GL)] += V[SH::vo(lv, c, 0)];
            });
          }
          if constexpr (lv < LG) {
            sfor<0, ncart(lv)>([&](auto c_) {
              constexpr int c = decltype(c_)::value;
#pragma unroll
              for (int m = 1; m <= MR; ++m) pub_put(wb + c * MR + m - 1, V[SH::vo(lv, c, m)]);
            });
            wave_lds_sync();
          }
        });
      }
      __syncthreads();  // the stage is rewritten by the next batch
    }
    // ---- sum the groups, contracted [e0|f0] into W (e-major), HRR, digest
    sfor<0, NGT>([&](auto k_) {
      constexpr int k = decltype(k_)::value;
      TV tot = acc[k];
      if constexpr (NGRP > 1) {
#pragma unroll
        for (int g = 1; g < NGRP; ++g) tot += __shfl(acc[k], g * NS + sidx);
      }
      if (active && grp == 0 && ns >= SH::SL) {
        const int ks = sidx - noff(SH::SL);
        const int tt = KL ? (k * NF + ks) : (ks * NF + k);
        W[tt] = (double)tot;
      }
    });
    __syncthreads();
    hrr_w<CB, CK>(W, cd, s, bra, ket, lane);
    if constexpr (LG <= 3)
      digest_w<CB, CK>(W + cd.out_base, s, bi, ki, bra, ket, g1, g2, g3, qb, lane);
    else
      digest_w<CB, CK>(W + cd.out_base, s, bi, ki, bra, ket, g1, g2, g3, quartet_blocks(s, bi, ki, g1, g2, g3), lane);
    __syncthreads();
  }
  if (lane == 0 && prims) atomicAdd(nprim, prims);
}

// lane side: the pair class with the lower total angular momentum
template <int CB, int CK>
constexpr bool lane_ket() {
  return class_la(CK) + class_lb(CK) < class_la(CB) + class_lb(CB);
}

template <int CB, int CK, int OP, typename TV>
void launch_lane_t(const CoopDev &cd, const SegLaunch &L) {
  if (L.nq_hint == 0) return;
  constexpr bool KL = lane_ket<CB, CK>();
  using SH = LaneShape<CB, CK, KL>;
  // up to 64 one-wave blocks per CU (measured 1-3% faster than 32)
  const int64_t blocks = seg_grid(L, L.nq_hint, 256 * 64);
  constexpr size_t lds = SH::template lds_bytes<TV>();
  hipLaunchKernelGGL((eri_lane_kernel<CB, CK, OP, KL, TV>), dim3((unsigned)blocks), dim3(64), lds, L.stream,
                     L.sys, L.nsys, L.seg, cd, L.list, L.nprim);
}

// HRR region the kernel reserves (doubles), for the host-side table check
template <int CB, int CK>
constexpr int lane_hrr_capacity() {
  return 2 * LaneShape<CB, CK, lane_ket<CB, CK>()>::hrr_r();
}

}  // namespace hfx

#define HFX_LANE_UNIT(CB, CK)                                                                        \
  namespace hfx {                                                                                    \
  void launch_eri_lane_r##CB##CK(int op, bool f32, const CoopDev &cd, const SegLaunch &L) {         \
    if (f32) {                                                                                       \
      if (op == 0)                                                                                   \
        launch_lane_t<CB, CK, 0, float>(cd, L);                                                      \
      else                                                                                           \
        launch_lane_t<CB, CK, 1, float>(cd, L);                                                      \
    } else {                                                                                         \
      if (op == 0)                                                                                   \
        launch_lane_t<CB, CK, 0, double>(cd, L);                                                     \
      else                                                                                           \
        launch_lane_t<CB, CK, 1, double>(cd, L);                                                     \
    }                                                                                                \
  }                                                                                                  \
  int lane_hrr_capacity_r##CB##CK() { return lane_hrr_capacity<CB, CK>(); }                          \
  }
