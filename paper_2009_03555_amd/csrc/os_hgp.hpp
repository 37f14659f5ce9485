// Contracted shell-quartet ERIs by the Obara-Saika vertical recursion
// (Obara & Saika, J. Chem. Phys. 84, 3963 (1986)) in the Head-Gordon-Pople
// arrangement (J. Chem. Phys. 89, 5777 (1988)): VRR to [e0|f0] per primitive
// quartet, sum over primitives, horizontal transfer to (ab|cd) once per
// contracted quartet.  All index arithmetic is resolved at compile time
// (one instantiation per angular-momentum class), so every intermediate has a
// fixed register slot.
//
// Operators (the paper's full-range ERI and Eq. ERI-SR): the auxiliary ladder
// is G_m = F_m(T) for 1/r and G_m = F_m(T) - s^(m+1/2) F_m(sT),
// s = omega^2 / (omega^2 + rho), for erfc(omega r)/r, from the Gaussian
// transform of erf(omega r)/r; the recursion coefficients do not change.
#pragma once
#include "hfx_common.hpp"

namespace hfx {

// 1/sqrt(x) for a positive normal x: the hardware estimate refined by two
// Newton steps y <- y + y (1 - x y^2) / 2, each squaring the relative error,
// to within a few ulp.  One of these replaces a correctly rounded division
// and a square root (about twice the instructions) where a primitive
// quartet needs both 1/x and 1/sqrt(x).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}

// ----------------------------------------------------------------- Boys
// F_m(T), m = 0..L.  T < 40: eight-term Taylor series of F_L about the
// nearest grid point (|dT| <= 1/32, truncation < 3e-17 relative), then the
// downward recursion F_m = (2T F_{m+1} + e^-T) / (2m+1), with e^-T from the
// tabulated e^-T_i times an eight-term series of e^-dT.  T >= 40: F_0 =
// sqrt(pi/T)/2 (erf(sqrt T) = 1 to 1e-18) and the upward recursion
// F_{m+1} = ((2m+1) F_m - e^-T) / (2T), stable for T > m + 1/2.
template <int L>
__device__ __forceinline__ void boys_eval(double T, const double *__restrict__ tab, double *F) {
  if (T < kBoysTmax) {
    int i = __double2int_rn(T * 16.0);
    double d = T - (double)i * kBoysStep;
    const double *row = tab + i * kBoysCols;
    double x = -d;
    double f = row[L + 7];
    f = fma(f, x * (1.0 / 7.0), row[L + 6]);
    f = fma(f, x * (1.0 / 6.0), row[L + 5]);
    f = fma(f, x * (1.0 / 5.0), row[L + 4]);
    f = fma(f, x * (1.0 / 4.0), row[L + 3]);
    f = fma(f, x * (1.0 / 3.0), row[L + 2]);
    f = fma(f, x * (1.0 / 2.0), row[L + 1]);
    f = fma(f, x, row[L]);
    F[L] = f;
    if constexpr (L > 0) {
      double e = 1.0;
      e = fma(e, x * (1.0 / 7.0), 1.0);
      e = fma(e, x * (1.0 / 6.0), 1.0);
      e = fma(e, x * (1.0 / 5.0), 1.0);
      e = fma(e, x * (1.0 / 4.0), 1.0);
      e = fma(e, x * (1.0 / 3.0), 1.0);
      e = fma(e, x * (1.0 / 2.0), 1.0);
      e = fma(e, x, 1.0);
      e *= row[16];
      double t2 = 2.0 * T;
#pragma unroll
      for (int m = L - 1; m >= 0; --m) F[m] = fma(t2, F[m + 1], e) * (1.0 / (2 * m + 1));
    }
  } else {
    const double y = rsqrt_nr(T);
    F[0] = 0.88622692545275801365 * y;  // (1/2) sqrt(pi / T)
    if constexpr (L > 0) {
      double e = exp(-T);
      double hr = 0.5 * (y * y);
#pragma unroll
      for (int m = 0; m < L; ++m) F[m + 1] = fma((double)(2 * m + 1), F[m], -e) * hr;
    }
  }
}

// Auxiliary ladder G_m (m = 0..L) times the common prefactor.
template <int L, int OP>
__device__ __forceinline__ void ladder(double T, double rho, double omega2, double pref,
                                       const double *__restrict__ tab, double *G) {
  boys_eval<L>(T, tab, G);
  if constexpr (OP == 1) {
    // s = omega^2 / (omega^2 + rho), sqrt(s) = omega / sqrt(omega^2 + rho)
    const double r = rsqrt_nr(omega2 + rho);
    double sp = sqrt(omega2) * r;
    const double s = omega2 * (r * r);
    double Fs[L + 1];
    boys_eval<L>(s * T, tab, Fs);
#pragma unroll
    for (int m = 0; m <= L; ++m) {
      G[m] = fma(-sp, Fs[m], G[m]);
      sp *= s;
    }
  }
#pragma unroll
  for (int m = 0; m <= L; ++m) G[m] *= pref;
}

// ------------------------------------------------------------- class traits
template <int LA_, int LB_, int LC_, int LD_>
struct Cls {
  static constexpr int LA = LA_, LB = LB_, LC = LC_, LD = LD_;
  static constexpr int EB = LA + LB, FK = LC + LD, L = EB + FK;
  static constexpr int NE = noff(EB + 1) - noff(LA);   // [e0| components, e in LA..EB
  static constexpr int NF = noff(FK + 1) - noff(LC);   // |f0] components, f in LC..FK
  static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
  static constexpr int NACC = NE * NF;
  static constexpr int NOUT = NA * NB * NC * ND;
};

// ------------------------------------------------------------------ VRR
// One primitive quartet: build [e0|f0]^(0) for e in [LA, EB], f in [LC, FK]
// from the ladder G[0..L] and add it to acc[NE][NF].
template <class C, typename T>
__device__ __forceinline__ void vrr_add(const T *G, const T *PA, const T *WP, const T *QC, const T *WQ,
                                        T o2z, T rz, T o2e, T re, T o2ze, T *acc) {
  constexpr int L = C::L, EB = C::EB, FK = C::FK, LA = C::LA, LC = C::LC;
  constexpr int NEA = noff(EB + 1);
  // stage 1: [e0|00]^(m), e = 0..EB, m = 0..L-e
  T S[L + 1][NEA];
  sfor<0, L + 1>([&](auto m_) { S[decltype(m_)::value][0] = G[decltype(m_)::value]; });
  sfor<1, EB + 1>([&](auto e_) {
    constexpr int e = decltype(e_)::value;
    sfor<0, ncart(e)>([&](auto c_) {
      constexpr int c = decltype(c_)::value;
      constexpr C3 v = cart_of(e, c);
      constexpr int i = dir_of(v);
      constexpr C3 v1 = sub1(v, i);
      constexpr int k = noff(e) + c;
      constexpr int k1 = noff(e - 1) + cidx(v1);
      constexpr int n1 = pw(v1, i);
      constexpr int k2 = n1 > 0 ? noff(e - 2) + cidx(sub1(v1, i)) : 0;
      sfor<0, L - e + 1>([&](auto m_) {
        constexpr int m = decltype(m_)::value;
        T r = PA[i] * S[m][k1] + WP[i] * S[m + 1][k1];
        if constexpr (n1 > 0) r += T(n1) * o2z * (S[m][k2] - rz * S[m + 1][k2]);
        S[m][k] = r;
      });
    });
  });
  if constexpr (FK == 0) {
    sfor<0, C::NE>([&](auto k_) {
      constexpr int k = decltype(k_)::value;
      acc[k] += S[0][noff(LA) + k];
    });
  } else {
    // stage 2: [e0|f0]^(m), f = 1..FK, m = 0..FK-f, e = max(0, LA-(FK-f))..EB
    constexpr int NFA = noff(FK + 1);
    T V[FK + 1][NEA][NFA];
    constexpr int elo0 = cmax(0, LA - FK);
    sfor<noff(elo0), NEA>([&](auto k_) {
      constexpr int k = decltype(k_)::value;
      sfor<0, FK + 1>([&](auto m_) { V[decltype(m_)::value][k][0] = S[decltype(m_)::value][k]; });
    });
    sfor<1, FK + 1>([&](auto f_) {
      constexpr int f = decltype(f_)::value;
      constexpr int elo = cmax(0, LA - (FK - f));
      sfor<0, ncart(f)>([&](auto d_) {
        constexpr int d = decltype(d_)::value;
        constexpr C3 w = cart_of(f, d);
        constexpr int i = dir_of(w);
        constexpr C3 w1 = sub1(w, i);
        constexpr int j = noff(f) + d;
        constexpr int j1 = noff(f - 1) + cidx(w1);
        constexpr int nf = pw(w1, i);
        constexpr int j2 = nf > 0 ? noff(f - 2) + cidx(sub1(w1, i)) : 0;
        sfor<noff(elo), NEA>([&](auto k_) {
          constexpr int k = decltype(k_)::value;
          constexpr int e = (k >= noff(1)) + (k >= noff(2)) + (k >= noff(3)) + (k >= noff(4)) +
                            (k >= noff(5)) + (k >= noff(6)) + (k >= noff(7)) + (k >= noff(8));
          constexpr C3 u = cart_of(e, k - noff(e));
          constexpr int ne = pw(u, i);
          constexpr int km = ne > 0 ? noff(e - 1) + cidx(sub1(u, i)) : 0;
          sfor<0, FK - f + 1>([&](auto m_) {
            constexpr int m = decltype(m_)::value;
            T r = QC[i] * V[m][k][j1] + WQ[i] * V[m + 1][k][j1];
            if constexpr (nf > 0) r += T(nf) * o2e * (V[m][k][j2] - re * V[m + 1][k][j2]);
            if constexpr (ne > 0) r += T(ne) * o2ze * V[m + 1][km][j1];
            V[m][k][j] = r;
          });
        });
      });
    });
    sfor<0, C::NE>([&](auto ke_) {
      constexpr int ke = decltype(ke_)::value;
      sfor<0, C::NF>([&](auto kf_) {
        constexpr int kf = decltype(kf_)::value;
        acc[ke * C::NF + kf] += V[0][noff(LA) + ke][noff(LC) + kf];
      });
    });
  }
}

// ------------------------------------------------------------------ HRR
// (a, b+1_i| = (a+1_i, b| + AB_i (a, b|, applied to the bra of acc[NE][NF]
// then to the ket, giving out[NA][NB][NC][ND].
template <class C>
__device__ __forceinline__ void hrr(const double *acc, const double *AB, const double *CD, double *out) {
  constexpr int LA = C::LA, LB = C::LB, LC = C::LC, LD = C::LD, EB = C::EB, FK = C::FK;
  constexpr int NF = C::NF;
  // bra: X[b][(a index over levels LA..EB-b)][b comp] for each f component
  constexpr int NAall = C::NE;  // a components, levels LA..EB
  double Y[C::NA * C::NB][NF];  // (ab|f]
  if constexpr (LB == 0) {
    sfor<0, C::NA>([&](auto a_) {
      sfor<0, NF>([&](auto f_) {
        Y[decltype(a_)::value][decltype(f_)::value] = acc[decltype(a_)::value * NF + decltype(f_)::value];
      });
    });
  } else {
    // level-by-level transfer, b = 1..LB
    double X[LB + 1][NAall][ncart(LB)][NF];
    sfor<0, NAall>([&](auto a_) {
      sfor<0, NF>([&](auto f_) {
        X[0][decltype(a_)::value][0][decltype(f_)::value] = acc[decltype(a_)::value * NF + decltype(f_)::value];
      });
    });
    sfor<1, LB + 1>([&](auto b_) {
      constexpr int b = decltype(b_)::value;
      sfor<0, ncart(b)>([&](auto cb_) {
        constexpr int cb = decltype(cb_)::value;
        constexpr C3 vb = cart_of(b, cb);
        constexpr int i = dir_of(vb);
        constexpr int cb1 = cidx(sub1(vb, i));
        // a levels LA..EB-b
        sfor<0, noff(EB - b + 1) - noff(LA)>([&](auto ka_) {
          constexpr int ka = decltype(ka_)::value;
          constexpr int aa = (ka + noff(LA) >= noff(1)) + (ka + noff(LA) >= noff(2)) +
                             (ka + noff(LA) >= noff(3)) + (ka + noff(LA) >= noff(4)) +
                             (ka + noff(LA) >= noff(5));
          constexpr C3 va = cart_of(aa, ka + noff(LA) - noff(aa));
          constexpr int kap = noff(aa + 1) + cidx(add1(va, i)) - noff(LA);
          sfor<0, NF>([&](auto f_) {
            constexpr int f = decltype(f_)::value;
            X[b][ka][cb][f] = X[b - 1][kap][cb1][f] + AB[i] * X[b - 1][ka][cb1][f];
          });
        });
      });
    });
    sfor<0, C::NA>([&](auto a_) {
      sfor<0, C::NB>([&](auto b_) {
        sfor<0, NF>([&](auto f_) {
          Y[decltype(a_)::value * C::NB + decltype(b_)::value][decltype(f_)::value] =
              X[LB][decltype(a_)::value][decltype(b_)::value][decltype(f_)::value];
        });
      });
    });
  }
  // ket
  if constexpr (LD == 0) {
    sfor<0, C::NA * C::NB>([&](auto ab_) {
      sfor<0, C::NC>([&](auto c_) {
        out[decltype(ab_)::value * C::NC + decltype(c_)::value] = Y[decltype(ab_)::value][decltype(c_)::value];
      });
    });
  } else {
    constexpr int NCall = NF;
    sfor<0, C::NA * C::NB>([&](auto ab_) {
      constexpr int ab = decltype(ab_)::value;
      double Z[LD + 1][NCall][ncart(LD)];
      sfor<0, NCall>([&](auto c_) { Z[0][decltype(c_)::value][0] = Y[ab][decltype(c_)::value]; });
      sfor<1, LD + 1>([&](auto d_) {
        constexpr int d = decltype(d_)::value;
        sfor<0, ncart(d)>([&](auto cd_) {
          constexpr int cd = decltype(cd_)::value;
          constexpr C3 vd = cart_of(d, cd);
          constexpr int i = dir_of(vd);
          constexpr int cd1 = cidx(sub1(vd, i));
          sfor<0, noff(FK - d + 1) - noff(LC)>([&](auto kc_) {
            constexpr int kc = decltype(kc_)::value;
            constexpr int cc = (kc + noff(LC) >= noff(1)) + (kc + noff(LC) >= noff(2)) +
                               (kc + noff(LC) >= noff(3)) + (kc + noff(LC) >= noff(4)) +
                               (kc + noff(LC) >= noff(5));
            constexpr C3 vc = cart_of(cc, kc + noff(LC) - noff(cc));
            constexpr int kcp = noff(cc + 1) + cidx(add1(vc, i)) - noff(LC);
            Z[d][kc][cd] = Z[d - 1][kcp][cd1] + CD[i] * Z[d - 1][kc][cd1];
          });
        });
      });
      sfor<0, C::NC>([&](auto c_) {
        sfor<0, C::ND>([&](auto d_) {
          out[(ab * C::NC + decltype(c_)::value) * C::ND + decltype(d_)::value] =
              Z[LD][decltype(c_)::value][decltype(d_)::value];
        });
      });
    });
  }
}

// ------------------------------------------------------- primitive loop
// Sum of [e0|f0] over the primitive quartets t = lane, lane+stride, ... of
// the nb x nk grid.  Ket centres are shifted by g (lattice translation).
// T is the type of the recursion and of the primitive sum: double, or float
// for the mixed-precision path (the ladder, including the Boys function, and
// the prefactor are always evaluated in double and rounded once).
// UNR: bra primitive iterations unrolled (2 keeps two in flight; measured
// per class, see the one-lane kernel)
template <class C, int OP, typename T = double, int UNR = 1>
__device__ __forceinline__ int prim_sum(const DevSys &s, const double *__restrict__ ppb, int nb,
                                        const double *__restrict__ ppk, int nk, double gx, double gy,
                                        double gz, int lane, int stride, T *acc, double thr = 0.0) {
  constexpr int L = C::L;
  int done = 0;
  if (nb <= 0) return 0;
  // ket primitive pairs lane, lane + stride, ..., each record read once; for
  // each, the bra primitive pairs it keeps.  Pair (ib, ik) is kept unless
  // k_bound < thr / b_bound: with both record lists sorted by descending
  // bound that is a prefix of the bra list for every ket pair (and of the ket
  // list for every bra pair: the same set the lane kernels count), so the
  // inner loop has a fixed trip count and its loads are the bra pair's
  // records, shared by the quartets of a wave that have the same bra pair.
  // (A wave's quartets share the bra pair and differ in the ket pair: with
  // the ket records in the inner loop, a wave streamed them from memory once
  // per bra primitive pair, 2.5-3.6 TB/s of HBM reads on the 64-atom diamond
  // cell; this order is 11-30% faster there.)
  for (int ik = lane; ik < nk; ik += stride) {
    const double *k = ppk + (int64_t)ik * kPP;
    const double kbnd = k[9];
    if (kbnd < thr / ppb[9]) break;
    const double eta = k[0];
    const double Qx = k[1] + gx, Qy = k[2] + gy, Qz = k[3] + gz;
    const T QC[3] = {(T)k[4], (T)k[5], (T)k[6]};
    const double kk = k[7];
    const T o2e = (T)k[8];
    int nbe = 0;
    {
      int hi = nb;
      while (nbe < hi) {
        const int mid = (nbe + hi) >> 1;
        if (kbnd < thr / ppb[(int64_t)mid * kPP + 9])
          hi = mid;
        else
          nbe = mid + 1;
      }
    }
    done += nbe;
#pragma unroll UNR
    for (int ib = 0; ib < nbe; ++ib) {
      const double *b = ppb + (int64_t)ib * kPP;
      const double zeta = b[0];
      const double rze = rsqrt_nr(zeta + eta);
      const double ize = rze * rze;
      const double rho = zeta * eta * ize;
      const double PQx = b[1] - Qx, PQy = b[2] - Qy, PQz = b[3] - Qz;
      const double T2 = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
      // 2 pi^(5/2) / (zeta eta sqrt(zeta + eta)) K_ab K_cd
      const double pref = b[7] * kk * rze;
      double G[L + 1];
      ladder<L, OP>(T2, rho, s.omega2, pref, s.boys, G);
      const double fe = eta * ize, fz = zeta * ize;
      T Gt[L + 1];
#pragma unroll
      for (int m = 0; m <= L; ++m) Gt[m] = (T)G[m];
      const T PA[3] = {(T)b[4], (T)b[5], (T)b[6]};
      const T WP[3] = {(T)(-fe * PQx), (T)(-fe * PQy), (T)(-fe * PQz)};
      const T WQ[3] = {(T)(fz * PQx), (T)(fz * PQy), (T)(fz * PQz)};
      // rho/zeta = eta/(zeta+eta), rho/eta = zeta/(zeta+eta)
      vrr_add<C, T>(Gt, PA, WP, QC, WQ, (T)b[8], (T)fe, o2e, (T)fz, (T)(0.5 * ize), acc);
    }
  }
  return done;
}

}  // namespace hfx
