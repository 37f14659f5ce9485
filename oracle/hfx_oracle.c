/*
 * Plain FP64 CPU oracle for the screened exchange build.  TEST INFRASTRUCTURE
 * ONLY: tests, the smoke check and the CPU-baseline leg of the benchmark call
 * it; the product path never does.  It shares no code with the HIP path.
 *
 * What it computes (paper, Background section):
 *   Eq. (H-HFX) without the -1/2 factor,
 *     K^G_{mu,lambda} = sum_{nu,sigma} sum_{N,H} D^{H-N}_{nu,sigma}
 *                        (mu^0 nu^N | lambda^G sigma^H),
 *   with mu in the home cell, over contracted Cartesian GTO shells, for the
 *   full-range Coulomb kernel 1/r (the full-range ERI definition) or the
 *   short-range kernel erfc(omega r)/r (Eq. ERI-SR).
 *   Shell-pair lists keep pairs whose centres are within the pair cutoff
 *   (distance screening); one sparse block pattern is shared by D and K
 *   (Parallelization section, sparse replicated D/K; Table 1).
 *   An ordered shell quartet is kept iff (Q_IJ * Q_KL) * P_scr > tau with
 *   Q_IJ = sqrt(max |(ij|ij)|) (Eq. schwarz) and
 *   P_scr = max(|P^IK|, |P^IL|, |P^JK|, |P^JL|) (Eq. dmscreening), each P the
 *   largest |D| of the Cartesian block, absent blocks counting 0.
 *
 * How (the paper names no integral method; these are textbook routes chosen
 * to differ from the GPU's Obara-Saika/Head-Gordon-Pople recursions):
 *   - McMurchie-Davidson: Hermite expansion coefficients E^{ij}_t and Hermite
 *     Coulomb integrals R^n_{tuv} (Helgaker, Jorgensen, Olsen, "Molecular
 *     Electronic-Structure Theory", ch. 9).
 *   - Boys function F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt in long double:
 *     the convergent series exp(-T) sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1))
 *     plus downward recursion for T < 45; erf closed form for F_0 plus upward
 *     recursion otherwise.
 *   - Attenuated kernels through the Gaussian transform of erf(omega r)/r:
 *     the ladder F_m(T) becomes s^{m+1/2} F_m(sT), s = omega^2/(omega^2+rho);
 *     erfc = Coulomb - erf.
 *   - Plain loop over every ordered quartet of each requested K block; no
 *     permutational symmetry, no compaction, no primitive screening.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXL 2
#define OR_MAXLT (4 * OR_MAXL)
#define OR_MAXCART 6

enum { OR_COULOMB = 0, OR_ERFC = 1, OR_ERF = 2 };

/* ------------------------------------------------------------------ Boys */
/* F_m(T) for m = 0..mmax into F (long double). */
void oracle_boys_ld(int mmax, long double T, long double *F) {
  if (T < 45.0L) {
    long double et = expl(-T);
    /* series for F_mmax */
    long double term = 1.0L / (2 * mmax + 1);
    long double sum = term;
    for (int k = 1; k < 100000; ++k) {
      term *= 2.0L * T / (2 * mmax + 2 * k + 1);
      sum += term;
      if (term < sum * 1e-21L) break;
    }
    F[mmax] = et * sum;
    for (int m = mmax - 1; m >= 0; --m) F[m] = (2.0L * T * F[m + 1] + et) / (2 * m + 1);
  } else {
    long double et = expl(-T);
    long double st = sqrtl(T);
    F[0] = 0.5L * sqrtl(3.14159265358979323846264338327950288L / T) * erfl(st);
    for (int m = 0; m < mmax; ++m) F[m + 1] = ((2 * m + 1) * F[m] - et) / (2.0L * T);
  }
}

void oracle_boys(int mmax, double T, double *out) {
  long double F[64];
  oracle_boys_ld(mmax, (long double)T, F);
  for (int m = 0; m <= mmax; ++m) out[m] = (double)F[m];
}

/* Operator ladder G_m, m = 0..mmax, for exponent rho and T = rho |PQ|^2. */
static void op_ladder(int op, double omega, int mmax, double rho, double T, long double *G) {
  long double F[OR_MAXLT + 2];
  if (op == OR_COULOMB) {
    oracle_boys_ld(mmax, T, F);
    for (int m = 0; m <= mmax; ++m) G[m] = F[m];
    return;
  }
  long double w2 = (long double)omega * omega;
  long double s = w2 / (w2 + rho);
  long double Fs[OR_MAXLT + 2];
  oracle_boys_ld(mmax, s * T, Fs);
  long double sp = sqrtl(s);
  if (op == OR_ERF) {
    for (int m = 0; m <= mmax; ++m) { G[m] = sp * Fs[m]; sp *= s; }
    return;
  }
  oracle_boys_ld(mmax, T, F);
  for (int m = 0; m <= mmax; ++m) { G[m] = F[m] - sp * Fs[m]; sp *= s; }
}

void oracle_op_ladder(int op, double omega, int mmax, double rho, double T, double *out) {
  long double G[OR_MAXLT + 2];
  op_ladder(op, omega, mmax, rho, T, G);
  for (int m = 0; m <= mmax; ++m) out[m] = (double)G[m];
}

/* ------------------------------------------------------- normalisation */
static double dfact(int n) { /* (n)!! with (-1)!! = 1 */
  double r = 1.0;
  for (int k = n; k > 1; k -= 2) r *= k;
  return r;
}

/* Normalised contraction coefficients (primitive norm folded in), so that
 * the x^l Cartesian component of the contracted shell has unit self-overlap. */
void oracle_normalize(int l, int nprim, const double *ex, const double *c_raw, double *c_out) {
  const double pi = 3.14159265358979323846;
  double N[64];
  for (int k = 0; k < nprim; ++k)
    N[k] = pow(2.0 * ex[k] / pi, 0.75) * pow(4.0 * ex[k], 0.5 * l) / sqrt(dfact(2 * l - 1));
  double S = 0.0;
  for (int k = 0; k < nprim; ++k)
    for (int j = 0; j < nprim; ++j) {
      double p = ex[k] + ex[j];
      S += c_raw[k] * c_raw[j] * N[k] * N[j] * pow(pi / p, 1.5) * dfact(2 * l - 1) / pow(2.0 * p, l);
    }
  for (int k = 0; k < nprim; ++k) c_out[k] = c_raw[k] * N[k] / sqrt(S);
}

/* ---------------------------------------------------- Cartesian indexing */
static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

/* exponents of component k of shell l, lexicographic x before y before z */
static void cart_xyz(int l, int k, int *lx, int *ly, int *lz) {
  int idx = 0;
  for (int x = l; x >= 0; --x)
    for (int y = l - x; y >= 0; --y) {
      if (idx == k) { *lx = x; *ly = y; *lz = l - x - y; return; }
      ++idx;
    }
}

/* ------------------------------------------------ McMurchie-Davidson ERI */
typedef struct {
  double xyz[3];
  int l, nprim;
  const double *ex, *c; /* normalised coefficients */
} oshell;

/* E[i][j][t] for one Cartesian direction */
static void hermite_E(int la, int lb, double a, double b, double XA, double XB,
                      double E[OR_MAXL + 1][OR_MAXL + 1][2 * OR_MAXL + 2]) {
  double p = a + b;
  double mu = a * b / p;
  double XAB = XA - XB;
  double XPA = (a * XA + b * XB) / p - XA;
  double XPB = (a * XA + b * XB) / p - XB;
  memset(E, 0, sizeof(double) * (OR_MAXL + 1) * (OR_MAXL + 1) * (2 * OR_MAXL + 2));
  E[0][0][0] = exp(-mu * XAB * XAB);
  for (int i = 0; i <= la; ++i)
    for (int j = 0; j <= lb; ++j) {
      if (i == 0 && j == 0) continue;
      for (int t = 0; t <= i + j; ++t) {
        double v;
        if (i > 0) {
          v = XPA * E[i - 1][j][t];
          if (t > 0) v += E[i - 1][j][t - 1] / (2 * p);
          if (t + 1 <= i - 1 + j) v += (t + 1) * E[i - 1][j][t + 1];
        } else {
          v = XPB * E[i][j - 1][t];
          if (t > 0) v += E[i][j - 1][t - 1] / (2 * p);
          if (t + 1 <= i + j - 1) v += (t + 1) * E[i][j - 1][t + 1];
        }
        E[i][j][t] = v;
      }
    }
}

#define RD (OR_MAXLT + 1)
/* Contracted shell quartet, Cartesian, out[a][b][c][d] row-major. */
void oracle_eri_quartet(const oshell *A, const oshell *B, const oshell *C, const oshell *D,
                        int op, double omega, double *out) {
  const double pi = 3.14159265358979323846;
  int na = ncart(A->l), nb = ncart(B->l), nc = ncart(C->l), nd = ncart(D->l);
  int L = A->l + B->l + C->l + D->l;
  memset(out, 0, sizeof(double) * na * nb * nc * nd);
  int ax[OR_MAXCART][3], bx[OR_MAXCART][3], cx[OR_MAXCART][3], dx[OR_MAXCART][3];
  for (int k = 0; k < na; ++k) cart_xyz(A->l, k, &ax[k][0], &ax[k][1], &ax[k][2]);
  for (int k = 0; k < nb; ++k) cart_xyz(B->l, k, &bx[k][0], &bx[k][1], &bx[k][2]);
  for (int k = 0; k < nc; ++k) cart_xyz(C->l, k, &cx[k][0], &cx[k][1], &cx[k][2]);
  for (int k = 0; k < nd; ++k) cart_xyz(D->l, k, &dx[k][0], &dx[k][1], &dx[k][2]);
  static __thread double R[RD][RD][RD][RD];
  double Eab[3][OR_MAXL + 1][OR_MAXL + 1][2 * OR_MAXL + 2];
  double Ecd[3][OR_MAXL + 1][OR_MAXL + 1][2 * OR_MAXL + 2];
  for (int ia = 0; ia < A->nprim; ++ia)
    for (int ib = 0; ib < B->nprim; ++ib) {
      double a = A->ex[ia], b = B->ex[ib], p = a + b;
      double P[3];
      for (int k = 0; k < 3; ++k) {
        P[k] = (a * A->xyz[k] + b * B->xyz[k]) / p;
        hermite_E(A->l, B->l, a, b, A->xyz[k], B->xyz[k], Eab[k]);
      }
      for (int ic = 0; ic < C->nprim; ++ic)
        for (int id = 0; id < D->nprim; ++id) {
          double c = C->ex[ic], d = D->ex[id], q = c + d;
          double Q[3];
          for (int k = 0; k < 3; ++k) {
            Q[k] = (c * C->xyz[k] + d * D->xyz[k]) / q;
            hermite_E(C->l, D->l, c, d, C->xyz[k], D->xyz[k], Ecd[k]);
          }
          double rho = p * q / (p + q);
          double PQ[3] = {P[0] - Q[0], P[1] - Q[1], P[2] - Q[2]};
          double T = rho * (PQ[0] * PQ[0] + PQ[1] * PQ[1] + PQ[2] * PQ[2]);
          long double G[OR_MAXLT + 2];
          op_ladder(op, omega, L, rho, T, G);
          /* Hermite Coulomb integrals R^n_{tuv} */
          long double m2r = 1.0L;
          for (int n = 0; n <= L; ++n) { R[n][0][0][0] = (double)(m2r * G[n]); m2r *= -2.0L * rho; }
          for (int tot = 1; tot <= L; ++tot)
            for (int n = 0; n <= L - tot; ++n)
              for (int t = tot; t >= 0; --t)
                for (int u = tot - t; u >= 0; --u) {
                  int v = tot - t - u;
                  double r;
                  if (t > 0) {
                    r = PQ[0] * R[n + 1][t - 1][u][v];
                    if (t > 1) r += (t - 1) * R[n + 1][t - 2][u][v];
                  } else if (u > 0) {
                    r = PQ[1] * R[n + 1][t][u - 1][v];
                    if (u > 1) r += (u - 1) * R[n + 1][t][u - 2][v];
                  } else {
                    r = PQ[2] * R[n + 1][t][u][v - 1];
                    if (v > 1) r += (v - 1) * R[n + 1][t][u][v - 2];
                  }
                  R[n][t][u][v] = r;
                }
          double pref = 2.0 * pow(pi, 2.5) / (p * q * sqrt(p + q)) *
                        A->c[ia] * B->c[ib] * C->c[ic] * D->c[id];
          for (int i = 0; i < na; ++i)
            for (int j = 0; j < nb; ++j) {
              int ex0 = ax[i][0], ey0 = ax[i][1], ez0 = ax[i][2];
              int fx0 = bx[j][0], fy0 = bx[j][1], fz0 = bx[j][2];
              for (int k = 0; k < nc; ++k)
                for (int l = 0; l < nd; ++l) {
                  int gx = cx[k][0], gy = cx[k][1], gz = cx[k][2];
                  int hx = dx[l][0], hy = dx[l][1], hz = dx[l][2];
                  double s = 0.0;
                  for (int t = 0; t <= ex0 + fx0; ++t)
                    for (int u = 0; u <= ey0 + fy0; ++u)
                      for (int v = 0; v <= ez0 + fz0; ++v) {
                        double eab = Eab[0][ex0][fx0][t] * Eab[1][ey0][fy0][u] * Eab[2][ez0][fz0][v];
                        if (eab == 0.0) continue;
                        double inner = 0.0;
                        for (int tt = 0; tt <= gx + hx; ++tt)
                          for (int uu = 0; uu <= gy + hy; ++uu)
                            for (int vv = 0; vv <= gz + hz; ++vv) {
                              double ecd = Ecd[0][gx][hx][tt] * Ecd[1][gy][hy][uu] * Ecd[2][gz][hz][vv];
                              double sg = ((tt + uu + vv) & 1) ? -1.0 : 1.0;
                              inner += sg * ecd * R[0][t + tt][u + uu][v + vv];
                            }
                        s += eab * inner;
                      }
                  out[((i * nb + j) * nc + k) * nd + l] += pref * s;
                }
            }
        }
    }
}

/* Convenience for pins: one quartet from raw arrays (coefficients already
 * normalised by the caller or not - used as given). */
void oracle_eri_raw(const double *xyz4, const int *l4, const int *np4, const double *ex,
                    const double *c, int op, double omega, double *out) {
  oshell s[4];
  int off = 0;
  for (int k = 0; k < 4; ++k) {
    s[k].xyz[0] = xyz4[3 * k]; s[k].xyz[1] = xyz4[3 * k + 1]; s[k].xyz[2] = xyz4[3 * k + 2];
    s[k].l = l4[k]; s[k].nprim = np4[k]; s[k].ex = ex + off; s[k].c = c + off;
    off += np4[k];
  }
  oracle_eri_quartet(&s[0], &s[1], &s[2], &s[3], op, omega, out);
}

/* ------------------------------------------------- spherical transform */
/* T (rows: boundary functions, cols: Cartesian) for shell l.  d with
 * spherical != 0: real solid harmonics m = -2..2 over xx,xy,xz,yy,yz,zz. */
static int sph_T(int l, int spherical, double *T /* [5*6] max */) {
  int nc = ncart(l);
  if (l == 2 && spherical) {
    const double s3 = sqrt(3.0);
    double t[5][6] = {{0, s3, 0, 0, 0, 0},
                      {0, 0, 0, 0, s3, 0},
                      {-0.5, 0, 0, -0.5, 0, 1.0},
                      {0, 0, s3, 0, 0, 0},
                      {0.5 * s3, 0, 0, -0.5 * s3, 0, 0}};
    memcpy(T, t, sizeof(t));
    return 5;
  }
  memset(T, 0, sizeof(double) * nc * nc);
  for (int k = 0; k < nc; ++k) T[k * nc + k] = 1.0;
  return nc;
}

void oracle_sph_matrix(int l, int spherical, double *T, int *nrow) { *nrow = sph_T(l, spherical, T); }

/* ------------------------------------------------------------- system */
typedef struct {
  int n_atoms, n_shells;
  double *xyz;      /* atoms */
  int *sh_atom, *sh_l, *sh_np, *sh_off;
  double *ex, *c;   /* normalised */
  int periodic;
  double lat[9];
  double cutoff;
  int op;
  double omega, tau;
  int spherical;
  /* pattern */
  int64_t nblk;
  int32_t *blk;     /* [nblk][5]: I, J, n1, n2, n3 */
  int64_t *blk_off; /* offset of block values (boundary basis) */
  int64_t nnz;
  int64_t *row_start; /* [n_shells+1] */
  int imgR[3];
  int32_t *lut;     /* [I][J][img] -> block or -1 */
  int nimg;
  int64_t *partner;
  double *Q;        /* per block (pair) */
  double *Pmax;     /* per block */
  double *Dc;       /* Cartesian density, per block, offset blk_coff */
  int64_t *blk_coff;
  int64_t nnz_c;
} osys;

static int img_index(const osys *s, int n1, int n2, int n3) {
  if (abs(n1) > s->imgR[0] || abs(n2) > s->imgR[1] || abs(n3) > s->imgR[2]) return -1;
  return ((n1 + s->imgR[0]) * (2 * s->imgR[1] + 1) + (n2 + s->imgR[1])) * (2 * s->imgR[2] + 1) +
         (n3 + s->imgR[2]);
}

static int64_t find_block(const osys *s, int I, int J, int n1, int n2, int n3) {
  int k = img_index(s, n1, n2, n3);
  if (k < 0) return -1;
  return s->lut[((int64_t)I * s->n_shells + J) * s->nimg + k];
}

static void shell_center(const osys *s, int I, const int *n, double *out) {
  const double *r = s->xyz + 3 * s->sh_atom[I];
  for (int k = 0; k < 3; ++k) {
    out[k] = r[k];
    if (s->periodic) out[k] += n[0] * s->lat[k] + n[1] * s->lat[3 + k] + n[2] * s->lat[6 + k];
  }
}

static int nfb(const osys *s, int I) { /* boundary functions */
  int l = s->sh_l[I];
  return (l == 2 && s->spherical) ? 5 : ncart(l);
}

static int cmp5(const void *a, const void *b) {
  const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
  for (int k = 0; k < 5; ++k)
    if (x[k] != y[k]) return x[k] < y[k] ? -1 : 1;
  return 0;
}

static int lexpos(int n1, int n2, int n3) {
  return n1 > 0 || (n1 == 0 && (n2 > 0 || (n2 == 0 && n3 >= 0)));
}

void *oracle_create(int n_atoms, const double *xyz, int n_shells, const int *sh_atom, const int *sh_l,
                    const int *sh_np, const double *ex, const double *c_raw, const double *lattice,
                    double cutoff, int op, double omega, double tau, int spherical) {
  osys *s = (osys *)calloc(1, sizeof(osys));
  s->n_atoms = n_atoms;
  s->n_shells = n_shells;
  s->xyz = (double *)malloc(sizeof(double) * 3 * n_atoms);
  memcpy(s->xyz, xyz, sizeof(double) * 3 * n_atoms);
  s->sh_atom = (int *)malloc(sizeof(int) * n_shells);
  s->sh_l = (int *)malloc(sizeof(int) * n_shells);
  s->sh_np = (int *)malloc(sizeof(int) * n_shells);
  s->sh_off = (int *)malloc(sizeof(int) * (n_shells + 1));
  memcpy(s->sh_atom, sh_atom, sizeof(int) * n_shells);
  memcpy(s->sh_l, sh_l, sizeof(int) * n_shells);
  memcpy(s->sh_np, sh_np, sizeof(int) * n_shells);
  int tot = 0;
  for (int I = 0; I < n_shells; ++I) { s->sh_off[I] = tot; tot += sh_np[I]; }
  s->sh_off[n_shells] = tot;
  s->ex = (double *)malloc(sizeof(double) * tot);
  s->c = (double *)malloc(sizeof(double) * tot);
  memcpy(s->ex, ex, sizeof(double) * tot);
  for (int I = 0; I < n_shells; ++I)
    oracle_normalize(sh_l[I], sh_np[I], ex + s->sh_off[I], c_raw + s->sh_off[I], s->c + s->sh_off[I]);
  s->periodic = lattice != NULL;
  if (lattice) memcpy(s->lat, lattice, sizeof(double) * 9);
  s->cutoff = cutoff;
  s->op = op;
  s->omega = omega;
  s->tau = tau;
  s->spherical = spherical;

  /* image search box from the reciprocal vectors */
  int R[3] = {0, 0, 0};
  if (s->periodic) {
    const double *a = s->lat;
    double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                 a[2] * (a[3] * a[7] - a[4] * a[6]);
    /* reciprocal rows b_i with b_i . a_j = delta_ij: b = inv(A)^T */
    double inv[9] = {(a[4] * a[8] - a[5] * a[7]) / det, (a[2] * a[7] - a[1] * a[8]) / det,
                     (a[1] * a[5] - a[2] * a[4]) / det, (a[5] * a[6] - a[3] * a[8]) / det,
                     (a[0] * a[8] - a[2] * a[6]) / det, (a[2] * a[3] - a[0] * a[5]) / det,
                     (a[3] * a[7] - a[4] * a[6]) / det, (a[1] * a[6] - a[0] * a[7]) / det,
                     (a[0] * a[4] - a[1] * a[3]) / det};
    for (int i = 0; i < 3; ++i) {
      double bn = sqrt(inv[0 + i] * inv[0 + i] + inv[3 + i] * inv[3 + i] + inv[6 + i] * inv[6 + i]);
      R[i] = (int)ceil(cutoff * bn) + 2;
    }
  }
  /* pattern: (I, J, n) with |R_I - R_J - T_n| <= cutoff (all pairs if cutoff <= 0) */
  int64_t cap = 1024, nb = 0;
  int32_t *blk = (int32_t *)malloc(sizeof(int32_t) * 5 * cap);
  int maxn[3] = {0, 0, 0};
  for (int I = 0; I < n_shells; ++I)
    for (int J = 0; J < n_shells; ++J)
      for (int n1 = -R[0]; n1 <= R[0]; ++n1)
        for (int n2 = -R[1]; n2 <= R[1]; ++n2)
          for (int n3 = -R[2]; n3 <= R[2]; ++n3) {
            int n[3] = {n1, n2, n3}, z[3] = {0, 0, 0};
            double ri[3], rj[3];
            shell_center(s, I, z, ri);
            shell_center(s, J, n, rj);
            double d2 = (ri[0] - rj[0]) * (ri[0] - rj[0]) + (ri[1] - rj[1]) * (ri[1] - rj[1]) +
                        (ri[2] - rj[2]) * (ri[2] - rj[2]);
            if (cutoff > 0 && sqrt(d2) > cutoff) continue;
            if (nb == cap) { cap *= 2; blk = (int32_t *)realloc(blk, sizeof(int32_t) * 5 * cap); }
            int32_t *b = blk + 5 * nb++;
            b[0] = I; b[1] = J; b[2] = n1; b[3] = n2; b[4] = n3;
            for (int k = 0; k < 3; ++k) if (abs(n[k]) > maxn[k]) maxn[k] = abs(n[k]);
          }
  qsort(blk, nb, sizeof(int32_t) * 5, cmp5);
  s->nblk = nb;
  s->blk = blk;
  for (int k = 0; k < 3; ++k) s->imgR[k] = maxn[k];
  s->nimg = (2 * maxn[0] + 1) * (2 * maxn[1] + 1) * (2 * maxn[2] + 1);
  s->lut = (int32_t *)malloc(sizeof(int32_t) * (int64_t)n_shells * n_shells * s->nimg);
  for (int64_t k = 0; k < (int64_t)n_shells * n_shells * s->nimg; ++k) s->lut[k] = -1;
  s->blk_off = (int64_t *)malloc(sizeof(int64_t) * (nb + 1));
  s->blk_coff = (int64_t *)malloc(sizeof(int64_t) * (nb + 1));
  s->row_start = (int64_t *)calloc(n_shells + 1, sizeof(int64_t));
  int64_t off = 0, coff = 0;
  for (int64_t b = 0; b < nb; ++b) {
    int32_t *x = blk + 5 * b;
    s->lut[((int64_t)x[0] * n_shells + x[1]) * s->nimg + img_index(s, x[2], x[3], x[4])] = (int32_t)b;
    s->blk_off[b] = off;
    s->blk_coff[b] = coff;
    off += nfb(s, x[0]) * nfb(s, x[1]);
    coff += ncart(s->sh_l[x[0]]) * ncart(s->sh_l[x[1]]);
    s->row_start[x[0] + 1]++;
  }
  s->blk_off[nb] = off;
  s->blk_coff[nb] = coff;
  s->nnz = off;
  s->nnz_c = coff;
  for (int I = 0; I < n_shells; ++I) s->row_start[I + 1] += s->row_start[I];
  s->partner = (int64_t *)malloc(sizeof(int64_t) * nb);
  for (int64_t b = 0; b < nb; ++b) {
    int32_t *x = blk + 5 * b;
    s->partner[b] = find_block(s, x[1], x[0], -x[2], -x[3], -x[4]);
  }
  s->Q = (double *)calloc(nb, sizeof(double));
  s->Pmax = (double *)calloc(nb, sizeof(double));
  s->Dc = (double *)calloc(s->nnz_c > 0 ? s->nnz_c : 1, sizeof(double));
  return s;
}

void oracle_destroy(void *h) {
  osys *s = (osys *)h;
  if (!s) return;
  free(s->xyz); free(s->sh_atom); free(s->sh_l); free(s->sh_np); free(s->sh_off);
  free(s->ex); free(s->c); free(s->blk); free(s->blk_off); free(s->blk_coff);
  free(s->row_start); free(s->lut); free(s->partner); free(s->Q); free(s->Pmax); free(s->Dc);
  free(s);
}

int64_t oracle_n_blocks(void *h) { return ((osys *)h)->nblk; }
int64_t oracle_nnz(void *h) { return ((osys *)h)->nnz; }
void oracle_blocks(void *h, int32_t *out) {
  osys *s = (osys *)h;
  memcpy(out, s->blk, sizeof(int32_t) * 5 * s->nblk);
}
void oracle_block_offsets(void *h, int64_t *out) {
  osys *s = (osys *)h;
  memcpy(out, s->blk_off, sizeof(int64_t) * (s->nblk + 1));
}

static void make_shell(const osys *s, int I, const int *n, oshell *o) {
  shell_center(s, I, n, o->xyz);
  o->l = s->sh_l[I];
  o->nprim = s->sh_np[I];
  o->ex = s->ex + s->sh_off[I];
  o->c = s->c + s->sh_off[I];
}

static int is_canonical_block(const int32_t *x) {
  return x[0] < x[1] || (x[0] == x[1] && lexpos(x[2], x[3], x[4]));
}

/* Schwarz factors Q_IJ = sqrt(max |(ij|ij)|) for every block of the pattern,
 * computed on the canonical orientation of each pair. */
void oracle_schwarz(void *h, double *q_out) {
  osys *s = (osys *)h;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t b = 0; b < s->nblk; ++b) {
    const int32_t *x = s->blk + 5 * b;
    if (!is_canonical_block(x)) continue;
    int z[3] = {0, 0, 0}, n[3] = {x[2], x[3], x[4]};
    oshell A, B;
    make_shell(s, x[0], z, &A);
    make_shell(s, x[1], n, &B);
    int na = ncart(A.l), nb = ncart(B.l);
    double *e = (double *)malloc(sizeof(double) * na * nb * na * nb);
    oracle_eri_quartet(&A, &B, &A, &B, s->op, s->omega, e);
    double m = 0.0;
    for (int i = 0; i < na; ++i)
      for (int j = 0; j < nb; ++j) {
        double v = fabs(e[((i * nb + j) * na + i) * nb + j]);
        if (v > m) m = v;
      }
    free(e);
    s->Q[b] = sqrt(m);
  }
  for (int64_t b = 0; b < s->nblk; ++b)
    if (!is_canonical_block(s->blk + 5 * b)) s->Q[b] = s->Q[s->partner[b]];
  if (q_out) memcpy(q_out, s->Q, sizeof(double) * s->nblk);
}

/* Schwarz factors of the blocks of the given rows only (a K block (I, K, G)
 * needs the pairs of rows I and K), each from its own orientation; the
 * other blocks keep their value.  Same definition as oracle_schwarz. */
void oracle_schwarz_rows(void *h, int64_t nrows, const int32_t *rows, double *q_out) {
  osys *s = (osys *)h;
  for (int64_t k = 0; k < nrows; ++k) {
    const int I = rows[k];
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = s->row_start[I]; b < s->row_start[I + 1]; ++b) {
      const int32_t *x = s->blk + 5 * b;
      int z[3] = {0, 0, 0}, n[3] = {x[2], x[3], x[4]};
      oshell A, B;
      make_shell(s, x[0], z, &A);
      make_shell(s, x[1], n, &B);
      int na = ncart(A.l), nb = ncart(B.l);
      double *e = (double *)malloc(sizeof(double) * na * nb * na * nb);
      oracle_eri_quartet(&A, &B, &A, &B, s->op, s->omega, e);
      double m = 0.0;
      for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) {
          double v = fabs(e[((i * nb + j) * na + i) * nb + j]);
          if (v > m) m = v;
        }
      free(e);
      s->Q[b] = sqrt(m);
    }
  }
  if (q_out) memcpy(q_out, s->Q, sizeof(double) * s->nblk);
}

/* D in the boundary basis (pattern order) -> Cartesian blocks and P_max.
 * D_cart = T_I^T D T_J; P_max of the canonical block, copied to its partner. */
void oracle_set_density(void *h, const double *d, double *pmax_out) {
  osys *s = (osys *)h;
  double TI[36], TJ[36];
  for (int64_t b = 0; b < s->nblk; ++b) {
    const int32_t *x = s->blk + 5 * b;
    int ri = sph_T(s->sh_l[x[0]], s->spherical, TI);
    int rj = sph_T(s->sh_l[x[1]], s->spherical, TJ);
    int ci = ncart(s->sh_l[x[0]]), cj = ncart(s->sh_l[x[1]]);
    const double *db = d + s->blk_off[b];
    double *dc = s->Dc + s->blk_coff[b];
    for (int a = 0; a < ci; ++a)
      for (int c = 0; c < cj; ++c) {
        double v = 0.0;
        for (int m = 0; m < ri; ++m)
          for (int k = 0; k < rj; ++k) v += TI[m * ci + a] * db[m * rj + k] * TJ[k * cj + c];
        dc[a * cj + c] = v;
      }
  }
  for (int64_t b = 0; b < s->nblk; ++b) {
    const int32_t *x = s->blk + 5 * b;
    if (!is_canonical_block(x)) continue;
    int ci = ncart(s->sh_l[x[0]]), cj = ncart(s->sh_l[x[1]]);
    double m = 0.0;
    for (int k = 0; k < ci * cj; ++k) {
      double v = fabs(s->Dc[s->blk_coff[b] + k]);
      if (v > m) m = v;
    }
    s->Pmax[b] = m;
  }
  for (int64_t b = 0; b < s->nblk; ++b)
    if (!is_canonical_block(s->blk + 5 * b)) s->Pmax[b] = s->Pmax[s->partner[b]];
  if (pmax_out) memcpy(pmax_out, s->Pmax, sizeof(double) * s->nblk);
}

/* Cartesian density of the last oracle_set_density, for checking it:
 * coff_out[nblk + 1] block offsets, dc_out[nnz_c] values (either may be
 * NULL); returns nnz_c. */
int64_t oracle_density_cart(void *h, int64_t *coff_out, double *dc_out) {
  osys *s = (osys *)h;
  if (coff_out) memcpy(coff_out, s->blk_coff, sizeof(int64_t) * (s->nblk + 1));
  if (dc_out) memcpy(dc_out, s->Dc, sizeof(double) * s->nnz_c);
  return s->nnz_c;
}

/* Replace the block maxima the screening uses (e.g. by the larger of two
 * spin densities' maxima, so that one predicate serves both spins). */
void oracle_set_pmax(void *h, const double *pmax) {
  osys *s = (osys *)h;
  memcpy(s->Pmax, pmax, sizeof(double) * s->nblk);
}

static double pm(const osys *s, int I, int J, int n1, int n2, int n3) {
  int64_t b = find_block(s, I, J, n1, n2, n3);
  return b < 0 ? 0.0 : s->Pmax[b];
}

/* K for the requested blocks (indices into the pattern), boundary basis,
 * written to k_out at the blocks' own offsets (other entries untouched).
 * screened = 0 keeps every ordered quartet.  Returns the number of ordered
 * shell quartets whose integrals were evaluated. */
int64_t oracle_build_K(void *h, int64_t nreq, const int64_t *req, int screened, double *k_out) {
  osys *s = (osys *)h;
  int64_t evaluated = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : evaluated)
  for (int64_t r = 0; r < nreq; ++r) {
    int64_t kb = req[r];
    const int32_t *x = s->blk + 5 * kb;
    int I = x[0], K = x[1], G[3] = {x[2], x[3], x[4]};
    int ci = ncart(s->sh_l[I]), ck = ncart(s->sh_l[K]);
    double Kc[36];
    memset(Kc, 0, sizeof(Kc));
    double *eri = (double *)malloc(sizeof(double) * 1296);
    int z[3] = {0, 0, 0};
    for (int64_t pb = s->row_start[I]; pb < s->row_start[I + 1]; ++pb) {
      const int32_t *y = s->blk + 5 * pb; /* (I, J, N) */
      int J = y[1], N[3] = {y[2], y[3], y[4]};
      for (int64_t qb = s->row_start[K]; qb < s->row_start[K + 1]; ++qb) {
        const int32_t *w = s->blk + 5 * qb; /* (K, L, M) */
        int L = w[1], M[3] = {w[2], w[3], w[4]};
        int H[3] = {G[0] + M[0], G[1] + M[1], G[2] + M[2]};
        int64_t db = find_block(s, J, L, H[0] - N[0], H[1] - N[1], H[2] - N[2]);
        if (db < 0) continue; /* D^{H-N}_{JL} outside the pattern: zero */
        if (screened) {
          double pscr = pm(s, I, K, G[0], G[1], G[2]);
          double t = pm(s, I, L, H[0], H[1], H[2]);
          if (t > pscr) pscr = t;
          t = pm(s, J, K, G[0] - N[0], G[1] - N[1], G[2] - N[2]);
          if (t > pscr) pscr = t;
          t = pm(s, J, L, H[0] - N[0], H[1] - N[1], H[2] - N[2]);
          if (t > pscr) pscr = t;
          double bound = (s->Q[pb] * s->Q[qb]) * pscr;
          if (!(bound > s->tau)) continue;
        }
        oshell A, B, C, D;
        make_shell(s, I, z, &A);
        make_shell(s, J, N, &B);
        make_shell(s, K, G, &C);
        make_shell(s, L, H, &D);
        oracle_eri_quartet(&A, &B, &C, &D, s->op, s->omega, eri);
        ++evaluated;
        int nb = ncart(B.l), nd = ncart(D.l);
        const double *dc = s->Dc + s->blk_coff[db];
        for (int a = 0; a < ci; ++a)
          for (int c = 0; c < ck; ++c) {
            double acc = 0.0;
            for (int b = 0; b < nb; ++b)
              for (int d = 0; d < nd; ++d) acc += eri[((a * nb + b) * ck + c) * nd + d] * dc[b * nd + d];
            Kc[a * ck + c] += acc;
          }
      }
    }
    free(eri);
    double TI[36], TK[36];
    int ri = sph_T(s->sh_l[I], s->spherical, TI);
    int rk = sph_T(s->sh_l[K], s->spherical, TK);
    double *ko = k_out + s->blk_off[kb];
    for (int m = 0; m < ri; ++m)
      for (int n = 0; n < rk; ++n) {
        double v = 0.0;
        for (int a = 0; a < ci; ++a)
          for (int c = 0; c < ck; ++c) v += TI[m * ci + a] * Kc[a * ck + c] * TK[n * ck + c];
        ko[m * rk + n] = v;
      }
  }
  return evaluated;
}

/* K from the given ordered quartets only (rows of 13 ints as in
 * oracle_quartets), without screening: each row (I^0 J^N | K^G L^H) adds
 * (mu nu | lambda sigma) D^{H-N}_{nu sigma} to K^G_{mu lambda}, the plain
 * term of Eq. H-HFX; rows whose K or D block lies outside the pattern add
 * nothing.  k_out (pattern layout, nnz values) is overwritten.  Returns the
 * number of rows that contributed. */
int64_t oracle_K_from_quartets(void *h, int64_t n, const int32_t *rows, double *k_out) {
  osys *s = (osys *)h;
  double *kc = (double *)calloc((size_t)s->nnz_c, sizeof(double));
  int64_t used = 0;
  double eri[1296];
  for (int64_t r = 0; r < n; ++r) {
    const int32_t *o = rows + 13 * r;
    int I = o[0], J = o[1], N[3] = {o[2], o[3], o[4]};
    int K = o[5], L = o[6], M[3] = {o[7], o[8], o[9]};
    int G[3] = {o[10], o[11], o[12]};
    int H[3] = {G[0] + M[0], G[1] + M[1], G[2] + M[2]};
    int64_t kb = find_block(s, I, K, G[0], G[1], G[2]);
    int64_t db = find_block(s, J, L, H[0] - N[0], H[1] - N[1], H[2] - N[2]);
    if (kb < 0 || db < 0) continue;
    int z[3] = {0, 0, 0};
    oshell A, B, C, D;
    make_shell(s, I, z, &A);
    make_shell(s, J, N, &B);
    make_shell(s, K, G, &C);
    make_shell(s, L, H, &D);
    oracle_eri_quartet(&A, &B, &C, &D, s->op, s->omega, eri);
    int na = ncart(A.l), nb = ncart(B.l), nc = ncart(C.l), nd = ncart(D.l);
    const double *dc = s->Dc + s->blk_coff[db];
    double *ko = kc + s->blk_coff[kb];
    for (int a = 0; a < na; ++a)
      for (int c = 0; c < nc; ++c) {
        double acc = 0.0;
        for (int b = 0; b < nb; ++b)
          for (int d = 0; d < nd; ++d) acc += eri[((a * nb + b) * nc + c) * nd + d] * dc[b * nd + d];
        ko[a * nc + c] += acc;
      }
    ++used;
  }
  for (int64_t kb = 0; kb < s->nblk; ++kb) {
    const int32_t *x = s->blk + 5 * kb;
    int I = x[0], K = x[1];
    int ci = ncart(s->sh_l[I]), ck = ncart(s->sh_l[K]);
    double TI[36], TK[36];
    int ri = sph_T(s->sh_l[I], s->spherical, TI);
    int rk = sph_T(s->sh_l[K], s->spherical, TK);
    const double *kcb = kc + s->blk_coff[kb];
    double *ko = k_out + s->blk_off[kb];
    for (int m = 0; m < ri; ++m)
      for (int q = 0; q < rk; ++q) {
        double v = 0.0;
        for (int a = 0; a < ci; ++a)
          for (int c = 0; c < ck; ++c) v += TI[m * ci + a] * kcb[a * ck + c] * TK[q * ck + c];
        ko[m * rk + q] = v;
      }
  }
  free(kc);
  return used;
}

/* Ordered quartets (I^0 J^N | K^G L^H) kept by the predicate, for bra and
 * ket pairs in the pattern and ket translations G in the box |G_i| <= gR
 * (G = 0 for molecules).  Row r of out_i holds 13 ints
 * (I, J, N1, N2, N3, K, L, M1, M2, M3, G1, G2, G3) with H = G + M; out_b[r]
 * is the bound (Q_IJ * Q_KL) * P_scr.  Writes at most cap rows and returns
 * the total count. */
/* Kept ordered quartets (I^0 J^N | K^G L^(G+M)) of the predicate of
 * Eq. schwarz and Eq. dmscreening, bra block pb over the nbra blocks in
 * bra_blocks (NULL: every block), ket block qb over every block, G in the
 * cube |G_i| <= gR (molecules: G = 0).  Rows of 13 ints (I, J, N, K, L, M,
 * G) and bounds, at most cap of them written; returns the count. */
int64_t oracle_quartets_bra(void *h, int gR, int64_t nbra, const int64_t *bra_blocks, int64_t cap,
                            int32_t *out_i, double *out_b) {
  osys *s = (osys *)h;
  int64_t cnt = 0;
  const int64_t nb = bra_blocks ? nbra : s->nblk;
  for (int64_t ib = 0; ib < nb; ++ib) {
    const int64_t pb = bra_blocks ? bra_blocks[ib] : ib;
    const int32_t *y = s->blk + 5 * pb;
    int I = y[0], J = y[1], N[3] = {y[2], y[3], y[4]};
    for (int64_t qb = 0; qb < s->nblk; ++qb) {
      const int32_t *w = s->blk + 5 * qb;
      int K = w[0], L = w[1], M[3] = {w[2], w[3], w[4]};
      int r0 = s->periodic ? gR : 0;
      for (int g1 = -r0; g1 <= r0; ++g1)
        for (int g2 = -r0; g2 <= r0; ++g2)
          for (int g3 = -r0; g3 <= r0; ++g3) {
            int G[3] = {g1, g2, g3};
            int H[3] = {G[0] + M[0], G[1] + M[1], G[2] + M[2]};
            double pscr = pm(s, I, K, G[0], G[1], G[2]);
            double t = pm(s, I, L, H[0], H[1], H[2]);
            if (t > pscr) pscr = t;
            t = pm(s, J, K, G[0] - N[0], G[1] - N[1], G[2] - N[2]);
            if (t > pscr) pscr = t;
            t = pm(s, J, L, H[0] - N[0], H[1] - N[1], H[2] - N[2]);
            if (t > pscr) pscr = t;
            double bound = (s->Q[pb] * s->Q[qb]) * pscr;
            if (!(bound > s->tau)) continue;
            if (cnt < cap) {
              int32_t *o = out_i + 13 * cnt;
              o[0] = I; o[1] = J; o[2] = N[0]; o[3] = N[1]; o[4] = N[2];
              o[5] = K; o[6] = L; o[7] = M[0]; o[8] = M[1]; o[9] = M[2];
              o[10] = G[0]; o[11] = G[1]; o[12] = G[2];
              out_b[cnt] = bound;
            }
            ++cnt;
          }
    }
  }
  return cnt;
}

int64_t oracle_quartets(void *h, int gR, int64_t cap, int32_t *out_i, double *out_b) {
  return oracle_quartets_bra(h, gR, 0, NULL, cap, out_i, out_b);
}

/* Replace the Schwarz factors (one per block) the screening uses, e.g. by
 * another implementation's, to compare the quartet selection alone. */
void oracle_set_q(void *h, const double *q) {
  osys *s = (osys *)h;
  memcpy(s->Q, q, sizeof(double) * s->nblk);
}

/* Evaluate the given ordered quartets (rows of 13 ints as in
 * oracle_quartets) one by one - contracted Cartesian integrals plus the K
 * contraction with the D block - without screening.  Used to time the
 * oracle on a sample of a workload.  Returns the number evaluated; *checksum
 * receives the sum of the contributions (keeps the work observable). */
int64_t oracle_eval_quartets(void *h, int64_t n, const int32_t *rows, double *checksum) {
  osys *s = (osys *)h;
  double total = 0.0;
  int64_t done = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(+ : total, done)
  for (int64_t r = 0; r < n; ++r) {
    const int32_t *o = rows + 13 * r;
    int I = o[0], J = o[1], N[3] = {o[2], o[3], o[4]};
    int K = o[5], L = o[6], M[3] = {o[7], o[8], o[9]};
    int G[3] = {o[10], o[11], o[12]};
    int H[3] = {G[0] + M[0], G[1] + M[1], G[2] + M[2]};
    int z[3] = {0, 0, 0};
    oshell A, B, C, D;
    make_shell(s, I, z, &A);
    make_shell(s, J, N, &B);
    make_shell(s, K, G, &C);
    make_shell(s, L, H, &D);
    double eri[1296];
    oracle_eri_quartet(&A, &B, &C, &D, s->op, s->omega, eri);
    int64_t db = find_block(s, J, L, H[0] - N[0], H[1] - N[1], H[2] - N[2]);
    int na = ncart(A.l), nb = ncart(B.l), nc = ncart(C.l), nd = ncart(D.l);
    double acc = 0.0;
    if (db >= 0) {
      const double *dc = s->Dc + s->blk_coff[db];
      for (int a = 0; a < na; ++a)
        for (int c = 0; c < nc; ++c)
          for (int b = 0; b < nb; ++b)
            for (int d = 0; d < nd; ++d) acc += eri[((a * nb + b) * nc + c) * nd + d] * dc[b * nd + d];
    }
    total += acc;
    done += 1;
  }
  if (checksum) *checksum = total;
  return done;
}
