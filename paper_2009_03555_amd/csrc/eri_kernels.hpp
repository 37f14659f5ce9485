// ERI + digest kernels and Schwarz-diagonal kernels, one instantiation per
// angular-momentum class.  Included by eri_r<cb><ck>.hip (one translation
// unit per class region, compiled in parallel).
#pragma once
#include "launchers.hpp"
#include "os_hgp.hpp"

namespace hfx {

// Primitive iterations (inner loop) kept in flight by the one-lane kernel,
// per class: two where measured faster on the 64-atom diamond cell ((ds|ps)
// 5%, (dp|ss) 11%); elsewhere the unrolled loop's registers cost more (up to
// 45% slower)
constexpr int prim_unroll(int cb, int ck) {
  const int r = region_of(cb, ck);
  return (r == region_of(3, 1) || r == region_of(4, 0)) ? 2 : 1;
}

// FP64 classes whose one-lane kernel takes a wave's quartets one plan at a
// time with the plan index in a scalar register (see eri_digest_kernel):
// measured 2-18% faster on the 64-atom diamond cell ((ps|ps) 10%, (pp|ss)
// 4%, (pp|pp) 5%, (ds|pp) 18%, (dp|ss) 7%, (dd|ps) 2%); (ds|ss), (ds|ps)
// and (dp|ds) were 3-6% slower with it (register allocation), the others
// within 1%
constexpr bool plan_scalar(int cb, int ck) {
  const int r = region_of(cb, ck);
  return r == region_of(1, 1) || r == region_of(2, 0) || r == region_of(2, 2) || r == region_of(3, 2) ||
         r == region_of(4, 0) || r == region_of(5, 1);
}

// ----------------------------------------------------------------- digest
// The four "row-first" exchange contributions of one unique quartet
// (A^0 B^nB | C^G D^(G+nD)) with weight w; K = K4 + K4^T is formed later.
// Block indices: AC = (A,C,G), AD = (A,D,G+nD), BC = (B,C,G-nB),
// BD = (B,D,G+nD-nB); absent blocks (-1) drop their terms.
//   K[AC][a][c] += w sum_bd v D[BD][b][d]      K[BC][b][c] += w sum_ad v D[AD][a][d]
//   K[AD][a][d] += w sum_bc v D[BC][b][c]      K[BD][b][d] += w sum_ac v D[AC][a][c]
// A collinear-spin build digests the same integrals once per spin density.
template <class C>
__device__ __forceinline__ void digest(const DevSys &s, int bAC, int bAD, int bBC, int bBD, const double *v,
                                       double w, const double *__restrict__ Dc0, double *__restrict__ K40) {
  constexpr int NA = C::NA, NB = C::NB, NC = C::NC, ND = C::ND;
  auto V = [&](int a, int b, int c, int d) { return v[((a * NB + b) * NC + c) * ND + d]; };
  for (int sp = 0; sp < s.nspin; ++sp) {
  const double *__restrict__ Dc = Dc0 + sp * s.spin_stride;
  double *__restrict__ K4 = K40 + sp * s.spin_stride;
  if (bAC >= 0 && bBD >= 0) {
    const double *D = Dc + s.blk_coff[bBD];
    double dv[NB * ND];
#pragma unroll
    for (int k = 0; k < NB * ND; ++k) dv[k] = D[k];
    double *K = K4 + s.blk_coff[bAC];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int d = 0; d < ND; ++d) acc = fma(V(a, b, c, d), dv[b * ND + d], acc);
        unsafeAtomicAdd(K + a * NC + c, w * acc);
      }
  }
  if (bBC >= 0 && bAD >= 0) {
    const double *D = Dc + s.blk_coff[bAD];
    double dv[NA * ND];
#pragma unroll
    for (int k = 0; k < NA * ND; ++k) dv[k] = D[k];
    double *K = K4 + s.blk_coff[bBC];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
          for (int d = 0; d < ND; ++d) acc = fma(V(a, b, c, d), dv[a * ND + d], acc);
        unsafeAtomicAdd(K + b * NC + c, w * acc);
      }
  }
  if (bAD >= 0 && bBC >= 0) {
    const double *D = Dc + s.blk_coff[bBC];
    double dv[NB * NC];
#pragma unroll
    for (int k = 0; k < NB * NC; ++k) dv[k] = D[k];
    double *K = K4 + s.blk_coff[bAD];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int c = 0; c < NC; ++c) acc = fma(V(a, b, c, d), dv[b * NC + c], acc);
        unsafeAtomicAdd(K + a * ND + d, w * acc);
      }
  }
  if (bBD >= 0 && bAC >= 0) {
    const double *D = Dc + s.blk_coff[bAC];
    double dv[NA * NC];
#pragma unroll
    for (int k = 0; k < NA * NC; ++k) dv[k] = D[k];
    double *K = K4 + s.blk_coff[bBD];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
          for (int c = 0; c < NC; ++c) acc = fma(V(a, b, c, d), dv[a * NC + c], acc);
        unsafeAtomicAdd(K + b * ND + d, w * acc);
      }
  }
  }
}

// --------------------------------------------------------- ERI + digest
// One lane per unique quartet of the class segment (grid-stride loop).  The
// segment [seg[0], seg[nsys]) of the fused list holds the class's quartets of
// nsys plans (plan i: [seg[i], seg[i+1])); bounds are read on the device so
// the launch does not depend on host-side counts.
// Waves per SIMD asked of the one-lane kernel: one more than its registers
// give by themselves for (ps|ps) (3) and (ps|ss) (4), measured 10% and 3%
// faster on the 64-atom diamond cell despite a few spilled registers; no
// bound elsewhere
template <int CB, int CK>
constexpr int reg_waves() {
  return (CB == 1 && CK == 1) ? 3 : ((CB == 1 && CK == 0) ? 4 : 1);
}

template <int CB, int CK, int OP, typename TV>
__global__ __attribute__((amdgpu_flat_work_group_size(1, 256), amdgpu_waves_per_eu(reg_waves<CB, CK>()))) void
eri_digest_kernel(const DevSys *__restrict__ sys, int nsys,
                                                         const int64_t *__restrict__ seg,
                                                         const uint64_t *__restrict__ list,
                                                         unsigned long long *__restrict__ nprim) {
  using C = Cls<class_la(CB), class_lb(CB), class_la(CK), class_lb(CK)>;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  const int64_t q0 = seg[0], q1 = seg[nsys];
  unsigned long long prims = 0;
  int pl = 0;  // plan of the previous quartet
  for (int64_t qi = q0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; qi < q1; qi += nthreads) {
    pl = nsys > 1 ? plan_of_hint(seg, nsys, qi, pl) : 0;
    // With plan_scalar, the lanes of a wave take their quartets one plan at
    // a time: the first remaining lane's plan index, a scalar, selects the
    // lanes of that plan, so the plan's fields come from scalar loads
    // (indexed by the per-lane plan they are vector loads, on separate
    // builds too).  A wave almost always holds one plan, and then this runs
    // once.  Both copies of pl pass through an empty volatile asm: each pass
    // reads them afresh (the scalar comes from the lanes still active), and
    // the scalar, being defined first, is the one the optimiser keeps where
    // the two are equal.
    constexpr bool kScalarPlan = plan_scalar(CB, CK) && sizeof(TV) == 8;
    for (;;) {
    int pw = pl;
    if constexpr (kScalarPlan) {
      int pv = pl;
      asm volatile("" : "+v"(pv));
      pw = __builtin_amdgcn_readfirstlane(pv);
      int pc = pl;
      asm volatile("" : "+v"(pc));
      if (pc != pw) continue;
    }
    const DevSys &s = sys[pw];
    const double *__restrict__ Dc = s.Dc;
    double *__restrict__ K4 = s.K4;
    const uint64_t q = list[qi];
    const int bra = (int)(q & 0xFFFFFFull);
    const int ket = (int)((q >> 24) & 0xFFFFFFull);
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
    const QuartetBlocks qb = quartet_blocks(s, bi, ki, g1, g2, g3);
    TV acct[C::NACC];
#pragma unroll
    for (int k = 0; k < C::NACC; ++k) acct[k] = (TV)0;
    prims += (unsigned long long)prim_sum<C, OP, TV, prim_unroll(CB, CK)>(s, s.pp + (int64_t)bpp.x * kPP, bpp.y,
                                                     s.pp + (int64_t)kpp.x * kPP, kpp.y, gx, gy, gz, 0, 1, acct,
                                                     prim_threshold(qb.pscr));
    double acc[C::NACC];
#pragma unroll
    for (int k = 0; k < C::NACC; ++k) acc[k] = (double)acct[k];
    const double *bg = s.pr_geom + (int64_t)bra * 8;
    const double *kg = s.pr_geom + (int64_t)ket * 8;
    double AB[3] = {bg[0], bg[1], bg[2]};
    double CD[3] = {kg[0], kg[1], kg[2]};
    double out[C::NOUT];
    hrr<C>(acc, AB, CD, out);
    double w = 1.0;
    if (bi.w & 1) w *= 0.5;
    if (ki.w & 1) w *= 0.5;
    if (bra == ket && g1 == 0 && g2 == 0 && g3 == 0) w *= 0.5;
    digest<C>(s, qb.AC, qb.AD, qb.BC, qb.BD, out, w, Dc, K4);
    break;
    }
  }
  // one counter update per thread
  prims += __shfl_xor(prims, 1);
  prims += __shfl_xor(prims, 2);
  prims += __shfl_xor(prims, 4);
  prims += __shfl_xor(prims, 8);
  prims += __shfl_xor(prims, 16);
  prims += __shfl_xor(prims, 32);
  if ((threadIdx.x & 63) == 0 && prims) atomicAdd(nprim, prims);
}

// ------------------------------------------------------------ Schwarz
// Q_p = sqrt(max_{a,b} |(ab|ab)|) over all primitive pairs of pair p.
template <int CB, int OP>
__global__ __launch_bounds__(128) void schwarz_kernel(DevSys s, int p0, int p1) {
  using C = Cls<class_la(CB), class_lb(CB), class_la(CB), class_lb(CB)>;
  const int p = p0 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (p >= p1) return;
  const int2 pp = s.pr_pp[p];
  const int n = s.pr_npp[p];
  double acc[C::NACC];
#pragma unroll
  for (int k = 0; k < C::NACC; ++k) acc[k] = 0.0;
  const double *b = s.pp + (int64_t)pp.x * kPP;
  prim_sum<C, OP>(s, b, n, b, n, 0.0, 0.0, 0.0, 0, 1, acc);
  const double *g = s.pr_geom + (int64_t)p * 8;
  double AB[3] = {g[0], g[1], g[2]};
  double out[C::NOUT];
  hrr<C>(acc, AB, AB, out);
  double m = 0.0;
#pragma unroll
  for (int a = 0; a < C::NA; ++a)
#pragma unroll
    for (int bb = 0; bb < C::NB; ++bb) m = fmax(m, fabs(out[((a * C::NB + bb) * C::NA + a) * C::NB + bb]));
  s.pr_Q[p] = sqrt(m);
}

// ------------------------------------------------------------ launchers
// nq_hint: quartets in the segment if known on the host (sizes the grid),
// or -1 (graph capture: a fixed grid that drains any count)
template <int CB, int CK, int OP, typename TV = double>
void launch_eri_t(const SegLaunch &L) {
  if (L.nq_hint == 0) return;
  // one-wave blocks (measured 0.5-3% faster per class than four-wave
  // blocks on the 64-atom diamond cell: finer placement at one or two waves
  // per SIMD).  Known count: one thread per quartet up to 256 * 256 blocks
  // (4M threads); graph replays (count unknown on the host): 256 * 32
  // blocks that stride
  const int threads = 64;
  const int64_t need = L.nq_hint > 0 ? (L.nq_hint + threads - 1) / threads : -1;
  const int64_t blocks = seg_grid(L, need, need > 0 ? 256 * 256 : 256 * 32);
  hipLaunchKernelGGL((eri_digest_kernel<CB, CK, OP, TV>), dim3((unsigned)blocks), dim3(threads), 0, L.stream,
                     L.sys, L.nsys, L.seg, L.list, L.nprim);
}

template <int CB, int OP>
void launch_schwarz_t(const DevSys &s, int p0, int p1, hipStream_t st) {
  if (p1 <= p0) return;
  const int threads = 128;
  hipLaunchKernelGGL((schwarz_kernel<CB, OP>), dim3((p1 - p0 + threads - 1) / threads), dim3(threads), 0, st, s,
                     p0, p1);
}

}  // namespace hfx

// Instantiate the launchers of one class region (bra class CB, ket class
// CK <= CB) in this translation unit; the diagonal unit (CK == CB) also holds
// the Schwarz kernels of pair class CB.
#define HFX_ERI_UNIT(CB, CK)                                                                         \
  namespace hfx {                                                                                    \
  void launch_eri_r##CB##CK(int op, const SegLaunch &L) {                                           \
    if (op == 0)                                                                                     \
      launch_eri_t<CB, CK, 0>(L);                                                                    \
    else                                                                                             \
      launch_eri_t<CB, CK, 1>(L);                                                                    \
  }                                                                                                  \
  }

// FP32-recursion variant of the region (mixed precision)
#define HFX_ERI_F32_UNIT(CB, CK)                                                                     \
  namespace hfx {                                                                                    \
  void launch_eri_f32_r##CB##CK(int op, const SegLaunch &L) {                                       \
    if (op == 0)                                                                                     \
      launch_eri_t<CB, CK, 0, float>(L);                                                             \
    else                                                                                             \
      launch_eri_t<CB, CK, 1, float>(L);                                                             \
  }                                                                                                  \
  }

#define HFX_SCHWARZ_UNIT(CB)                                                                         \
  namespace hfx {                                                                                    \
  void launch_schwarz_c##CB(int op, const DevSys &s, int p0, int p1, hipStream_t st) {              \
    if (op == 0)                                                                                     \
      launch_schwarz_t<CB, 0>(s, p0, p1, st);                                                        \
    else                                                                                             \
      launch_schwarz_t<CB, 1>(s, p0, p1, st);                                                        \
  }                                                                                                  \
  }
