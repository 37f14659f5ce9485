// Wave-cooperative ERI + digest kernel for high angular-momentum classes
// (see coop.hpp).  Per class, the level structure of the VRR is known at
// compile time, so each lane keeps its share of the VRR op list in registers
// for the whole launch and every level is pure LDS traffic plus FMAs.
#pragma once
#include "coop.hpp"
#include "launchers.hpp"
#include "os_hgp.hpp"
#include "eri_wave.hpp"

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
  int *pfx = reinterpret_cast<int *>(stage + kCoopBatch * kCoopStage);
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
    QuartetBlocks qb{-1, -1, -1, -1, 0.0};
    double thr = 0.0;  // the Schwarz mode sums every primitive quartet
    if constexpr (MODE == 0) {
      qb = quartet_blocks(s, bi, ki, g1, g2, g3);
      thr = prim_threshold(qb.pscr);
    }
    const int n = prim_prefix(pfx, ppb, bpp.y, ppk, kpp.y, thr, lane);
    prims += (unsigned long long)n;
    __syncthreads();
    double acc[SH64::SLOTS];
#pragma unroll
    for (int k = 0; k < SH64::SLOTS; ++k) acc[k] = 0.0;

    for (int t0 = 0; t0 < n; t0 += kCoopBatch) {
      stage_prims<L, OP>(stage, lane, kCoopBatch, t0, n, pfx, bpp.y, ppb, ppk, gx, gy, gz, s);
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
    if constexpr (MODE == 1) {
      schwarz_from_w<CB>(W, cd, s, bra, lane);
    } else {
      hrr_w<CB, CK>(W, cd, s, bra, ket, lane);
      digest_w<CB, CK>(W + cd.out_base, s, bi, ki, bra, ket, g1, g2, g3, qb, lane);
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
  const int64_t blocks = seg_grid(L, L.nq_hint, 256 * 32);
  const size_t lds = ((size_t)P * (cd.nw + 1) + (size_t)kCoopBatch * kCoopStage) * sizeof(double) +
                     kPfxInts * sizeof(int);
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
  const size_t lds = ((size_t)P * (cd.nw + 1) + (size_t)kCoopBatch * kCoopStage) * sizeof(double) +
                     kPfxInts * sizeof(int);
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
