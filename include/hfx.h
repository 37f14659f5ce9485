/*
 * hfx.h - C ABI of the MI355X screened exchange-matrix builder.
 *
 * The library evaluates screened contracted shell-quartet electron repulsion
 * integrals (ERIs) over Cartesian Gaussian shells (s, p, d) and contracts them
 * with a sparse density matrix D into the sparse exchange matrix K, following
 * the paper's Background section:
 *
 *   Eq. (H-HFX) without its -1/2 factor,
 *     K^G_{mu,lambda} = sum_{nu,sigma} sum_{N,H} D^{H-N}_{nu,sigma}
 *                        (mu^0 nu^N | lambda^G sigma^H),
 *   mu in the home cell, N, G, H lattice translations (molecules: all 0);
 *   kernel 1/|r-r'| (full-range ERI) or erfc(omega|r-r'|)/|r-r'| (Eq. ERI-SR);
 *   8-fold permutational symmetry with lattice translations (the permutation
 *   relations after Eq. ERI-SR) - each unique quartet is evaluated once;
 *   shell pairs preselected by distance and Schwarz factors (Eq. schwarz);
 *   quartets kept iff (Q_IJ * Q_KL) * P_scr > tau with
 *   P_scr = max(|P^IK|max, |P^IL|max, |P^JK|max, |P^JL|max) (Eq. dmscreening);
 *   D and K stored in one shared replicated sparse block format (the sparse
 *   format of both matrices in the Parallelization section, Table 1), with
 *   the sparse-to-dense index transform done twice per quartet (Algorithm 4).
 *
 * Conventions
 *   - Units: bohr, bohr^-2.  Lattice rows a1, a2, a3.
 *   - Cartesian component order within a shell: lexicographic, x before y
 *     before z (d: xx, xy, xz, yy, yz, zz), each component normalised like
 *     x^l.  With spherical_d != 0 the boundary basis of d shells is the five
 *     real solid harmonics m = -2..2 (sqrt3 xy, sqrt3 yz, zz-(xx+yy)/2,
 *     sqrt3 xz, sqrt3/2 (xx-yy)); integrals and screening are Cartesian,
 *     D_cart = T^T D T and K = T K_cart T^T at the boundary.
 *   - D must be symmetric: D^n_{ij} = D^{-n}_{ji} (a real density matrix).
 *   - Pattern: block (I, J, n) couples home-cell shell I with shell J
 *     translated by n, present iff |R_I - R_J - T_n| <= pair_cutoff (all
 *     (I, J, 0) for a molecule without cutoff).  Blocks are sorted by
 *     (I, J, n1, n2, n3); values row-major nfunc(I) x nfunc(J) at
 *     hfx_block.offset.  D entries outside the pattern are taken as zero and
 *     K outside the pattern is not formed.
 *   - Every call returns an hfx_status; no exception crosses the ABI.  On
 *     failure hfx_last_error() returns a thread-local message.
 *   - A plan is not thread-safe; distinct plans are independent.  All device
 *     work of a plan runs in order on the HIP stream given to hfx_plan.
 */
#ifndef HFX_H
#define HFX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HFX_OK = 0,
  HFX_ERR_INVALID = 1,     /* bad argument or system description */
  HFX_ERR_OOM = 2,         /* device allocation failed */
  HFX_ERR_DEVICE = 3,      /* HIP runtime error */
  HFX_ERR_STATE = 4,       /* call out of order, or destroyed plan */
  HFX_ERR_UNSUPPORTED = 5  /* outside the implemented range (l > 2, ...) */
} hfx_status;

typedef enum { HFX_OP_COULOMB = 0, HFX_OP_ERFC = 1 } hfx_operator;
typedef enum { HFX_FP64 = 0, HFX_MIXED = 1 } hfx_precision;

#define HFX_MAX_L 2
#define HFX_MAX_PRIM 8

/* flags for hfx_build_K */
#define HFX_SYNC 1u        /* synchronise the stream before returning */
#define HFX_TIMING 2u      /* record per-phase times into info (implies SYNC) */
#define HFX_GRAPH 4u       /* replay the build as a captured HIP graph (see below) */

typedef struct hfx_plan_s *hfx_plan_t;

/* System description.  All pointers are host memory, read during hfx_plan
 * only (the plan copies what it needs). */
typedef struct {
  int32_t n_atoms;
  const double *atom_xyz;     /* [n_atoms * 3] */
  int32_t n_shells;
  const int32_t *shell_atom;  /* [n_shells], 0 <= . < n_atoms */
  const int32_t *shell_l;     /* [n_shells], 0..HFX_MAX_L */
  const int32_t *shell_nprim; /* [n_shells], 1..HFX_MAX_PRIM */
  const double *prim_exp;     /* [sum nprim], > 0 */
  const double *prim_coef;    /* [sum nprim], raw; the plan normalises */
  const double *lattice;      /* [9] rows a1,a2,a3, or NULL for a molecule */
  double pair_cutoff;         /* bohr; <= 0: all pairs (molecules only) */
  int32_t op;                 /* hfx_operator */
  double omega;               /* bohr^-1, used iff op == HFX_OP_ERFC */
  double tau;                 /* keep a quartet iff bound > tau (>= 0) */
  int32_t precision;          /* hfx_precision */
  double fp32_cutoff;         /* HFX_MIXED: Q_IJ*Q_KL below this allows the FP32 path;
                                 classes whose FP32 kernel is no faster stay FP64:
                                 (ss|ss) (ps|ss) (ps|ps) (pp|ps) (ds|ss) (dd|ss), and
                                 (dd|dd), whose HRR amplifies FP32 rounding too much */
  int32_t spherical_d;        /* 1: five spherical d functions; 0: six Cartesian */
} hfx_system;

/* One pattern block (plan-owned array, valid until hfx_plan_destroy). */
typedef struct {
  int32_t I, J;
  int32_t img[3];
  int32_t pad;
  int64_t offset;             /* first value in the D/K arrays */
} hfx_block;

#define HFX_N_CLASSES 21

/* Optional per-build report (valid once the build's stream work is done). */
typedef struct {
  int64_t n_quartets;                     /* unique quartets kept by screening */
  int64_t n_quartets_class[HFX_N_CLASSES];
  int64_t n_prim_quartets;                /* primitive quartets evaluated */
  int64_t n_fp32_quartets;                /* quartets taken on the FP32 path */
  double flops;                           /* algorithmic FLOPs of the ERI phase */
  double ms_density, ms_screen, ms_eri, ms_finalize, ms_total; /* HFX_TIMING */
  double ms_class[HFX_N_CLASSES];         /* HFX_TIMING: ERI kernel time per class (0 for a
                                             chunked list, whose ERI time counts in ms_screen) */
  double flops_class[HFX_N_CLASSES];      /* algorithmic FLOPs per class */
  int64_t n_chunks;                       /* list chunks evaluated (0: every list whole) */
} hfx_build_info;

/* Device bytes hfx_plan would allocate for this system (its tables and its
 * own one-plan batch), plus the plan's share of a fused multi-plan batch,
 * excluding the per-build quartet lists (8 bytes per screened quartet,
 * reported in *list_bytes_per_quartet), the second-spin arrays of
 * hfx_build_K_spin and the library's per-device static arrays (the Boys
 * table, 87 KB, shared by all plans, and the allocation-free build's
 * scratch).  Validates like hfx_plan; allocates nothing on the device. */
hfx_status hfx_footprint(const hfx_system *sys, size_t *device_bytes, size_t *list_bytes_per_quartet);

/* Validate, normalise contractions, build the pattern, shell-pair and
 * primitive-pair tables and the block lookup, and upload them; the first
 * plan on a device also fills that device's Boys table.  stream:
 * hipStream_t (NULL = default stream).  *out receives the plan. */
hfx_status hfx_plan(const hfx_system *sys, void *stream, hfx_plan_t *out);

/* The shared D/K pattern.  *blocks points to plan-owned memory. */
hfx_status hfx_pattern(hfx_plan_t plan, int64_t *n_blocks, int64_t *nnz, const hfx_block **blocks);

/* Schwarz factors Q_IJ = sqrt(max_{i in I, j in J} |(ij|ij)|) with the
 * plan's operator, always FP64 (Eq. schwarz).  One value per pattern block
 * (a pair and its transpose share it).  q_host: NULL or host array of
 * n_blocks doubles to receive them.  *n_pairs: number of unique pairs. */
hfx_status hfx_schwarz(hfx_plan_t plan, double *q_host, int64_t *n_pairs);

/* One exchange build (Eq. H-HFX with the screening of Eq. schwarz and
 * Eq. dmscreening):
 * d_dev, k_dev are device arrays of nnz doubles in the pattern layout
 * (caller-owned).  K is overwritten.  Runs hfx_schwarz first if it has not
 * run.  Asynchronous on the plan's stream unless HFX_SYNC, HFX_TIMING or
 * info is given.
 *
 * HFX_GRAPH: after one eager build has sized the quartet lists, the whole
 * build (density transform, screening, every ERI class, finalisation) is
 * captured once per (d_dev, k_dev) pair into a HIP graph with list capacity
 * 1.25x the last size, and replayed.  A replay whose screened list outgrows
 * that capacity is detected on the device and redone eagerly (the next call
 * captures again).  Graph builds synchronise the stream before returning.
 * HFX_TIMING takes precedence over HFX_GRAPH. */
hfx_status hfx_build_K(hfx_plan_t plan, const double *d_dev, double *k_dev, uint32_t flags,
                       hfx_build_info *info);

/* Progress of chunked builds: fn(user, list, chunk, quartets_done,
 * quartets_total) is called on the calling thread after the device has
 * finished each chunk of a chunked list (list 0: the FP64 list, 1: the FP32
 * list of mixed precision; chunk: chunks finished so far in this build;
 * quartets of this list up to the end of the chunk, and in the whole list).
 * Setting it makes chunked builds wait for each chunk before screening the
 * next.  fn = NULL turns the reports off.  Fused multi-plan builds report to
 * the first plan's function. */
typedef void (*hfx_progress_fn)(void *user, int32_t list, int64_t chunk, int64_t quartets_done,
                                int64_t quartets_total);
hfx_status hfx_set_progress(hfx_plan_t plan, hfx_progress_fn fn, void *user);

/* Collinear spin: the exchange matrix of each spin density,
 * K^s_{mu nu} = sum_{lambda sigma} (mu lambda|nu sigma) D^s_{lambda sigma},
 * s = alpha, beta - Eq. H-HFX applied per spin, the spin-polarised form of
 * the Kohn-Sham equations the Background section writes for the
 * unpolarised case.  Every unique quartet's integrals are evaluated once and
 * digested into both K's.  One quartet list serves both spins: P_max of a
 * block is the larger of the two densities' block maxima (Eq. dmscreening
 * over both spins), so each K^s keeps every term a separate build of D^s
 * keeps, and possibly a few more of bound at most tau.  D and K arrays as
 * for hfx_build_K (caller-owned, nnz doubles each); flags and info as for
 * hfx_build_K (info: counts of the shared evaluation; flops include both
 * digests).  The first call allocates the plan's second-spin arrays. */
hfx_status hfx_build_K_spin(hfx_plan_t plan, const double *d_alpha, const double *d_beta, double *k_alpha,
                            double *k_beta, uint32_t flags, hfx_build_info *info);

/* Hartree-Fock exchange part of the Hamiltonian at k-points, from the
 * real-space exchange matrix of a build (Background section: the Bloch sum
 * of the Hamiltonian, [H(k)]_{mu nu} = sum_R <chi_mu^0|H|chi_nu^R>
 * exp(i k.(R + r_nu - r_mu)), applied to Eq. H-HFX, whose HFX part carries
 * the factor -1/2; alpha is the fraction of exact exchange the functional
 * mixes in, 1/4 for HSE06 (its short-range HF term, with the erfc
 * operator), 1 for Hartree-Fock):
 *   H(k)_{mu nu} = -(alpha / 2) sum_G K^G_{mu nu} exp(i k.(T_G + r_nu - r_mu)),
 * r_mu the home-cell position of mu's atom, T_G the lattice vector of
 * pattern block (mu's shell, nu's shell, G).
 * k_dev: device array of nnz doubles, K in the pattern layout (as written by
 * hfx_build_K).  kpts_host: host array [nk][3] of Cartesian k-points
 * (bohr^-1).  h_dev: caller-owned device array of 2 * nk * nbf * nbf
 * doubles, written as nk dense complex matrices (real, imaginary
 * interleaved), row-major, rows and columns in the boundary basis of the
 * cell's functions (shell order; nbf = their number); entries of shell
 * pairs outside the pattern are zero.  A molecule has T_G = 0 (use k = 0).
 * Runs on the plan's stream and synchronises it before returning. */
hfx_status hfx_kspace(hfx_plan_t plan, const double *k_dev, int32_t nk, const double *kpts_host, double alpha,
                      double *h_dev);

/* Largest number of unique quartets a build of this plan holds in one
 * quartet list (8 bytes each; default 2^33, i.e. 64 GiB; 0 restores the
 * default).  A screened list longer than this is evaluated in chunks: the
 * screening work items (one bra pair against one ket class) are cut into
 * consecutive ranges whose quartets fit, and each range is filled and run
 * through the ERI kernels before the next overwrites the buffer - the
 * batched evaluation of Algorithm 4 on one device.  Results equal the
 * unchunked build up to the order of floating-point additions.  A single
 * work item larger than the limit fails with HFX_ERR_OOM.  Chunked builds
 * run eagerly (no HFX_GRAPH replay) and keep no whole list for hfx_export
 * or hfx_autotune.  Fused multi-plan builds use the smallest limit of their
 * plans. */
hfx_status hfx_set_list_limit(hfx_plan_t plan, int64_t max_quartets);

/* hfx_build_K without any device allocation, for callers that cannot
 * allocate (code running under HIP graph capture elsewhere, tight serving
 * loops, harnesses that forbid hipMalloc).  The build's work arrays
 * (screening counts and offsets, class-segment bounds, error flags,
 * primitive-quartet counters and the quartet list) live in the library's
 * static device array of 256 MiB, one per device, held until the process
 * ends; every list is evaluated in chunks of what that array's list part
 * holds (also bounded by hfx_set_list_limit).  Results equal hfx_build_K up
 * to the order of floating-point additions.  flags: 0 or HFX_SYNC
 * (HFX_TIMING and HFX_GRAPH are HFX_ERR_INVALID); info as for hfx_build_K.
 * HFX_ERR_INVALID if the plan's screening work items alone need more of
 * the array than it has beside a list of 65536 quartets.  Calls on one
 * device share its array: calls that overlap in time on one device (other
 * threads, other streams) race and must be serialised by the caller. */
hfx_status hfx_build_K_noalloc(hfx_plan_t plan, const double *d_dev, double *k_dev, uint32_t flags,
                               hfx_build_info *info);

/* Several plans (each with its own D and K, all on one device) in fused
 * launches: one screening pass and one ERI launch per class cover every
 * plan of one operator; plans of the two operators form two such groups.
 * Runs on the stream of the first plan of each group.  Results equal n
 * separate hfx_build_K calls.  The fused state is cached per plan list (and
 * dropped when one of its plans is destroyed); flags as for hfx_build_K;
 * info sums over all plans.  A plan may appear at most once. */
hfx_status hfx_build_K_multi(int32_t n, const hfx_plan_t *plans, const double *const *d_dev,
                             double *const *k_dev, uint32_t flags, hfx_build_info *info);

/* K from a caller-chosen subset of the unique quartets only (a shard of the
 * screened list, or a sample for verification): the same density transform,
 * ERI and digest kernels (the plan's kernel choices) and finalisation as
 * hfx_build_K, over the n quartets in quartets_host (host memory, the
 * encoding of hfx_export what = 1: bra pair | ket pair << 24 | translation
 * << 48, any order; duplicates are evaluated twice).  The quartet screening
 * predicate is not applied (the caller chose the quartets); the primitive-
 * quartet bound is, with P_scr from d_dev; a mixed-precision plan sends the
 * quartets below its FP32 cutoff to the FP32 kernels, as a build would.
 * Synchronous.  HFX_ERR_INVALID if
 * a pair index is out of range or a quartet's bra pair class is below its
 * ket pair class. */
hfx_status hfx_build_K_subset(hfx_plan_t plan, const double *d_dev, double *k_dev, const uint64_t *quartets_host,
                              int64_t n);

/* Screened quartet count of a build with density d_dev, without building:
 * density transform, P_max and the counting pass of the screening only.
 * n64: quartets of the FP64 list, n32: of the FP32 list (mixed precision,
 * else 0); the quartet lists of a build need 8 bytes per quartet.  For
 * admission control before the first build. */
hfx_status hfx_screen_count(hfx_plan_t plan, const double *d_dev, int64_t *n64, int64_t *n32);

/* Autotuner (project-written): for every quartet class of the plan's
 * current screened list, time each available ERI kernel variant (one-lane
 * register recursion, wave-cooperative LDS recursion, lane-per-component
 * recursion; for the FP32 list of mixed precision also their FP32 forms) at
 * several grid sizes on the first max_quartets quartets of the class (all if
 * <= 0), keep the fastest for later builds of this plan (and of fused
 * multi-plan builds it leads), then run one build into k_dev.  Costs roughly
 * two builds of the sampled prefixes.  report may be NULL. */
#define HFX_TUNE_MAX_CAND 12
typedef struct {
  int32_t variant; /* 0 register, 1 cooperative, 2 lane, 3 register FP32, 4 lane FP32 */
  int32_t fp32_list; /* 1: candidate for the FP32 list of mixed precision */
  int64_t max_blocks; /* grid cap of the candidate (0: the kernel's default) */
  double ms;          /* time of the sampled prefix */
} hfx_tune_candidate;
typedef struct {
  int32_t n_candidates[HFX_N_CLASSES];
  int64_t sample_quartets[HFX_N_CLASSES];    /* FP64 list prefix timed */
  int64_t sample_quartets32[HFX_N_CLASSES];  /* FP32 list prefix timed */
  int32_t chosen[HFX_N_CLASSES];    /* index into cand of the FP64-list choice, -1 if none timed */
  int32_t chosen32[HFX_N_CLASSES];  /* same for the FP32 list */
  hfx_tune_candidate cand[HFX_N_CLASSES][HFX_TUNE_MAX_CAND];
} hfx_tune_report;
hfx_status hfx_autotune(hfx_plan_t plan, const double *d_dev, double *k_dev, int64_t max_quartets,
                        hfx_tune_report *report);

/* Host copies of the last hfx_build_K's screening data, for verification:
 * what = 0: P_max per pattern block (n doubles, n = n_blocks);
 * what = 1: quartet list as uint64 (bra pair | ket pair << 24 | image << 48),
 *           n = number of quartets;
 * what = 2: unique pair table as int32 [n][6] (A, B, n1, n2, n3, class);
 * what = 3: Schwarz factor per unique pair (n doubles);
 * what = 5: mixed precision: the FP32-path quartet list (uint64, as what = 1;
 *           what = 1 then holds the FP64-path quartets).
 * With host == NULL only *n is set. */
hfx_status hfx_export(hfx_plan_t plan, int32_t what, void *host, int64_t *n);

hfx_status hfx_plan_destroy(hfx_plan_t plan);

/* NAO2GTO (Introduction and Background: numerical atomic orbitals with a
 * strict cutoff, each fitted by several GTOs so that the ERIs are
 * analytical): fit the radial function radial[i] = R(r[i]) of angular
 * momentum l on the grid r (n_r increasing points >= 0, host memory) by
 * f(r) = sum_k c_k r^l exp(-a_k r^2), k < n_gto, minimising
 * sum_i w_i (R(r_i) - f(r_i))^2 with w_i = r_i^2 dr_i (trapezoid weights of
 * the radial measure).  Coefficients by weighted linear least squares for
 * given exponents, log-exponents by Levenberg-Marquardt from an
 * even-tempered start spanning the grid.  exps_out, coefs_out: n_gto host
 * doubles, exponents ascending; coefficients raw (multiplying r^l e^{-a r^2};
 * hfx_plan normalises a contraction, so they enter hfx_system.prim_coef as
 * they are).  *rms_out (nullable): sqrt(objective / sum_i w_i R_i^2).
 * HFX_ERR_INVALID for l outside 0..HFX_MAX_L, n_gto outside
 * 1..HFX_MAX_PRIM, fewer than 2 n_gto + 2 points, a non-increasing grid or a
 * zero function.  Host only: needs no device. */
hfx_status hfx_nao2gto_fit(int32_t l, int32_t n_r, const double *r, const double *radial, int32_t n_gto,
                           double *exps_out, double *coefs_out, double *rms_out);

const char *hfx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HFX_H */
