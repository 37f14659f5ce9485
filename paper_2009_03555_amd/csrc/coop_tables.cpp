// Host-side generation of the cooperative kernels' op lists: the Obara-Saika
// VRR to [e0|f0] and the HGP HRR to (ab|cd), in the same order and with the
// same transfer directions as the compile-time recursions of os_hgp.hpp.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <tuple>

#include "coop.hpp"

namespace hfx {
namespace {

C3 cart_rt(int l, int c) { return cart_of(l, c); }
int level_of(int k) {  // level of a flattened component index over levels 0..
  int l = 0;
  while (noff(l + 1) <= k) ++l;
  return l;
}

uint4 make_op(int out, int a, int b, int c, int d, int e, int dir, int n, int ne) {
  auto chk = [](int v) {
    if (v < 0 || v > 0xFFFF) {
      std::fprintf(stderr, "coop op offset out of range\n");
      std::abort();
    }
    return (uint32_t)v;
  };
  uint4 o;
  o.x = chk(out) | (chk(a) << 16);
  o.y = chk(b) | (chk(c) << 16);
  o.z = chk(d) | (chk(e) << 16);
  o.w = (uint32_t)dir | ((uint32_t)n << 2) | ((uint32_t)ne << 6);
  return o;
}

}  // namespace

int coop_level_count(int cb, int ck, int lv) {
  const int LA = class_la(cb), LB = class_lb(cb), LC = class_la(ck), LD = class_lb(ck);
  const int EB = LA + LB, FK = LC + LD, L = EB + FK;
  if (lv < EB) return ncart(lv + 1) * (L - lv);
  const int f = lv - EB + 1;
  const int elo = cmax(0, LA - (FK - f));
  return ncart(f) * (noff(EB + 1) - noff(elo)) * (FK - f + 1);
}

void coop_build(int cb, int ck, int gl, CoopHost &h) {
  const int LA = class_la(cb), LB = class_lb(cb), LC = class_la(ck), LD = class_lb(ck);
  const int EB = LA + LB, FK = LC + LD, L = EB + FK;
  h = CoopHost();
  h.la = LA; h.lb = LB; h.lc = LC; h.ld = LD; h.L = L;
  const int NE = noff(EB + 1) - noff(LA), NF = noff(FK + 1) - noff(LC);
  const int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
  h.nacc = NE * NF;
  h.nout = NA * NB * NC * ND;

  // ---------------- VRR layout: S[e-comp k][m] (m = 0..L-e), then stage-2 nodes
  int next = 0;
  std::map<std::pair<int, int>, int> S;  // (k, m) -> offset; k flattened over levels 0..EB
  for (int e = 0; e <= EB; ++e)
    for (int c = 0; c < ncart(e); ++c)
      for (int m = 0; m <= L - e; ++m) S[{noff(e) + c, m}] = next++;
  std::map<std::tuple<int, int, int>, int> V;  // (k, j, m) for f >= 1; j flattened over f levels
  auto voff = [&](int k, int j, int m) -> int {
    if (j == 0) return S.at({k, m});
    return V.at(std::make_tuple(k, j, m));
  };
  for (int f = 1; f <= FK; ++f) {
    const int elo = cmax(0, LA - (FK - f));
    for (int d = 0; d < ncart(f); ++d)
      for (int k = noff(elo); k < noff(EB + 1); ++k)
        for (int m = 0; m <= FK - f; ++m) V[std::make_tuple(k, noff(f) + d, m)] = next++;
  }
  const int nw_vrr = next;
  // ---------------- VRR ops
  // stage 1, one level per e
  for (int e = 1; e <= EB; ++e) {
    int4 lv = make_int4((int)h.ops.size(), 0, kOpVrrBra, 0);
    for (int c = 0; c < ncart(e); ++c) {
      const C3 v = cart_rt(e, c);
      const int i = dir_of(v);
      const C3 v1 = sub1(v, i);
      const int k = noff(e) + c, k1 = noff(e - 1) + cidx(v1);
      const int n1 = pw(v1, i);
      const int k2 = n1 > 0 ? noff(e - 2) + cidx(sub1(v1, i)) : 0;
      for (int m = 0; m <= L - e; ++m) {
        const int cc = n1 > 0 ? S.at({k2, m}) : 0, dd = n1 > 0 ? S.at({k2, m + 1}) : 0;
        h.ops.push_back(make_op(S.at({k, m}), S.at({k1, m}), S.at({k1, m + 1}), cc, dd, 0, i, n1, 0));
      }
    }
    lv.y = (int)h.ops.size() - lv.x;
    h.levels.push_back(lv);
  }
  // stage 2, one level per f
  for (int f = 1; f <= FK; ++f) {
    const int elo = cmax(0, LA - (FK - f));
    int4 lv = make_int4((int)h.ops.size(), 0, kOpVrrKet, 0);
    for (int d = 0; d < ncart(f); ++d) {
      const C3 w = cart_rt(f, d);
      const int i = dir_of(w);
      const C3 w1 = sub1(w, i);
      const int j = noff(f) + d, j1 = noff(f - 1) + cidx(w1);
      const int nf = pw(w1, i);
      const int j2 = nf > 0 ? noff(f - 2) + cidx(sub1(w1, i)) : 0;
      for (int k = noff(elo); k < noff(EB + 1); ++k) {
        const int e = level_of(k);
        const C3 u = cart_rt(e, k - noff(e));
        const int ne = pw(u, i);
        const int km = ne > 0 ? noff(e - 1) + cidx(sub1(u, i)) : 0;
        for (int m = 0; m <= FK - f; ++m) {
          const int cc = nf > 0 ? voff(k, j2, m) : 0, dd = nf > 0 ? voff(k, j2, m + 1) : 0;
          const int ee = ne > 0 ? voff(km, j1, m + 1) : 0;
          h.ops.push_back(make_op(voff(k, j, m), voff(k, j1, m), voff(k, j1, m + 1), cc, dd, ee, i, nf, ne));
        }
      }
    }
    lv.y = (int)h.ops.size() - lv.x;
    h.levels.push_back(lv);
  }
  h.n_vrr_levels = (int)h.levels.size();
  // targets
  for (int ke = 0; ke < NE; ++ke)
    for (int kf = 0; kf < NF; ++kf) h.acc_off.push_back((uint16_t)voff(noff(LA) + ke, FK == 0 ? 0 : noff(LC) + kf, 0));

  // ---------------- HRR (ping-pong regions P = [0, R), Q = [R, 2R))
  // level sizes
  std::vector<int> sizes;
  sizes.push_back(NE * NF);
  for (int b = 1; b <= LB; ++b) sizes.push_back((noff(EB - b + 1) - noff(LA)) * ncart(b) * NF);
  for (int d = 1; d <= LD; ++d) sizes.push_back(NA * NB * (noff(FK - d + 1) - noff(LC)) * ncart(d));
  const int R = *std::max_element(sizes.begin(), sizes.end());
  int cur = 0;  // region of the current level
  auto base = [&](int r) { return r * R; };
  // X_b[ka][cb][f], ka over a-levels LA..EB-b
  for (int b = 1; b <= LB; ++b) {
    const int src = base(cur), dst = base(1 - cur);
    const int NAb = noff(EB - b + 1) - noff(LA), NAb1 = noff(EB - b + 2) - noff(LA);
    (void)NAb1;
    int4 lv = make_int4((int)h.ops.size(), 0, kOpHrrBra, 0);
    for (int cbb = 0; cbb < ncart(b); ++cbb) {
      const C3 vb = cart_rt(b, cbb);
      const int i = dir_of(vb);
      const int cb1 = cidx(sub1(vb, i));
      for (int ka = 0; ka < NAb; ++ka) {
        const int aa = level_of(ka + noff(LA));
        const C3 va = cart_rt(aa, ka + noff(LA) - noff(aa));
        const int kap = noff(aa + 1) + cidx(add1(va, i)) - noff(LA);
        for (int f = 0; f < NF; ++f) {
          const int out = dst + (ka * ncart(b) + cbb) * NF + f;
          const int a = src + (kap * ncart(b - 1) + cb1) * NF + f;
          const int bb = src + (ka * ncart(b - 1) + cb1) * NF + f;
          h.ops.push_back(make_op(out, a, bb, 0, 0, 0, i, 0, 0));
        }
      }
    }
    lv.y = (int)h.ops.size() - lv.x;
    h.levels.push_back(lv);
    cur = 1 - cur;
  }
  // after the bra: Y[ab][f] = X_LB[ka][cb][f] with ab = ka * NB + cb (natural)
  // Z_d[ab][kc][cd], kc over c-levels LC..FK-d
  for (int d = 1; d <= LD; ++d) {
    const int src = base(cur), dst = base(1 - cur);
    const int NCd = noff(FK - d + 1) - noff(LC), NCd1 = noff(FK - d + 2) - noff(LC);
    int4 lv = make_int4((int)h.ops.size(), 0, kOpHrrKet, 0);
    for (int ab = 0; ab < NA * NB; ++ab)
      for (int cdd = 0; cdd < ncart(d); ++cdd) {
        const C3 vd = cart_rt(d, cdd);
        const int i = dir_of(vd);
        const int cd1 = cidx(sub1(vd, i));
        for (int kc = 0; kc < NCd; ++kc) {
          const int cc = level_of(kc + noff(LC));
          const C3 vc = cart_rt(cc, kc + noff(LC) - noff(cc));
          const int kcp = noff(cc + 1) + cidx(add1(vc, i)) - noff(LC);
          const int out = dst + (ab * NCd + kc) * ncart(d) + cdd;
          const int a = src + (ab * NCd1 + kcp) * ncart(d - 1) + cd1;
          const int bb = src + (ab * NCd1 + kc) * ncart(d - 1) + cd1;
          h.ops.push_back(make_op(out, a, bb, 0, 0, 0, i, 0, 0));
        }
      }
    lv.y = (int)h.ops.size() - lv.x;
    h.levels.push_back(lv);
    cur = 1 - cur;
  }
  h.n_hrr_levels = (int)h.levels.size() - h.n_vrr_levels;
  h.out_base = base(cur);
  h.nw = std::max(nw_vrr, 2 * R);
  // register form of the VRR ops, level by level padded to a multiple of gl;
  // byte offsets are multiples of 8 and their low bits carry ne, n and dir.
  // Padding steps write the dummy slot nw and read slot 0.
  for (int lv = 0; lv < h.n_vrr_levels; ++lv) {
    const int first = h.levels[lv].x, cnt = h.levels[lv].y;
    const int padded = (cnt + gl - 1) / gl * gl;
    for (int it = 0; it < padded; ++it) {
      uint32_t out = h.nw, a = 0, c = 0, e = 0, dir = 0, n = 0, ne = 0;
      if (it < cnt) {
        const uint4 o = h.ops[first + it];
        out = o.x & 0xFFFF;
        a = o.x >> 16;
        const uint32_t b = o.y & 0xFFFF, d = o.z & 0xFFFF;
        c = o.y >> 16;
        e = o.z >> 16;
        dir = o.w & 3;
        n = (o.w >> 2) & 15;
        ne = (o.w >> 6) & 15;
        if (b != a + 1 || (n > 0 && d != c + 1) || n > 7 || ne > 7) {
          std::fprintf(stderr, "coop register op out of range\n");
          std::abort();
        }
      }
      if ((out + 1) * 8 > 0xFFFF || (a + 2) * 8 > 0xFFFF || (c + 2) * 8 > 0xFFFF || (e + 1) * 8 > 0xFFFF) {
        std::fprintf(stderr, "coop register op out of range\n");
        std::abort();
      }
      uint4 r;
      r.x = (out * 8 | ne) | ((a * 8 | n) << 16);
      r.y = (c * 8 | dir) | ((e * 8) << 16);
      r.z = 0;
      r.w = 0;
      h.vops.push_back(r);
    }
  }
  if (h.nw > 0xFFFF) {
    std::fprintf(stderr, "coop workspace too large\n");
    std::abort();
  }
}

}  // namespace hfx
