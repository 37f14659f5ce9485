// Wave-cooperative evaluation of high angular-momentum classes.
//
// For classes whose per-primitive-quartet recursion does not fit one lane's
// registers, one 64-lane wave evaluates one contracted quartet: the
// intermediates of the current primitive quartet live in LDS, each level of
// the Obara-Saika VRR (and, after the primitive sum, of the HGP HRR) is split
// over the lanes, and the contracted [e0|f0] targets are owned by the lanes in
// registers (target t by lane t mod 64).  The level structure is an op list
// generated on the host from the same recursion rules as the compile-time
// kernels in os_hgp.hpp (same transfer direction, same terms).
#pragma once
#include <stdint.h>

#include <vector>

#include "hfx_common.hpp"

namespace hfx {

// op kinds (one per level)
enum : int { kOpVrrBra = 1, kOpVrrKet = 2, kOpHrrBra = 3, kOpHrrKet = 4 };

// One recursion step, four 32-bit words:
//   x = out | a << 16, y = b | c << 16, z = d | e << 16,
//   w = dir | n << 2 | ne << 6
// VRR bra:  W[out] = PA[dir] W[a] + WP[dir] W[b] + n/(2 zeta) (W[c] - rho/zeta W[d])
// VRR ket:  W[out] = QC[dir] W[a] + WQ[dir] W[b] + n/(2 eta) (W[c] - rho/eta W[d])
//                    + ne/(2 (zeta+eta)) W[e]
// HRR bra:  W[out] = W[a] + AB[dir] W[b];   HRR ket: W[out] = W[a] + CD[dir] W[b]
struct CoopDev {
  const uint4 *ops;
  const uint4 *vops;        // VRR ops, register form: x = (8 out | ne) | (8 a | n) << 16, y = (8 c | dir) | 8 e << 16
  const int4 *levels;       // (first op, op count, kind, unused)
  const uint16_t *acc_off;  // W offset of target t after the VRR of one primitive quartet
  int n_vrr_levels, n_hrr_levels;
  int nacc, nout, nw, out_base;
  int na, nb, nc, nd;
};

struct CoopHost {
  int la = 0, lb = 0, lc = 0, ld = 0, L = 0;
  int nacc = 0, nout = 0, nw = 0, out_base = 0;
  std::vector<uint4> ops;
  std::vector<uint4> vops;
  std::vector<int4> levels;
  std::vector<uint16_t> acc_off;
  int n_vrr_levels = 0, n_hrr_levels = 0;
};

// primitive quartets evaluated side by side per wave (lane groups of 64/P)
__host__ __device__ constexpr int coop_parallel(int cb, int ck) {
  return (class_la(cb) + class_lb(cb) + class_la(ck) + class_lb(ck)) <= 5
             ? 4
             : ((class_la(cb) + class_lb(cb) + class_la(ck) + class_lb(ck)) <= 7 ? 2 : 1);
}

// host: build the op lists of class (cb, ck); the register-form VRR list of
// every level is padded to a multiple of gl with no-op steps that write a
// dummy slot at offset nw (so every lane runs every round)
void coop_build(int cb, int ck, int gl, CoopHost &out);

// classes with a cooperative kernel (bra class >= dp and total L >= 5)
__host__ __device__ constexpr bool coop_available(int cb, int ck) {
  return cb >= 4 && class_la(cb) + class_lb(cb) + class_la(ck) + class_lb(ck) >= 5;
}
// level sizes of the VRR op list (must equal the kernel's compile-time shape)
int coop_level_count(int cb, int ck, int lv);

// Schwarz factors of pair class cb (4 or 5) through the cooperative kernel of
// class (cb|cb); cd must be that class's tables
void launch_schwarz_coop(int cb, int op, const DevSys *sys1, const CoopDev &cd, int p0, int p1, hipStream_t st);

struct SegLaunch;
void launch_eri_coop(int cb, int ck, int op, const CoopDev &cd, const SegLaunch &L);

}  // namespace hfx
