/* Low-scaling GW hot path on MI355X (gfx950): C ABI of libgw.so.
 *
 * Method: Wilhelm, Golze, Talirz, Hutter, Pignedoli, "Towards GW calculations
 * on thousands of atoms", J. Phys. Chem. Lett. (2018), arXiv:2104.09857.
 * Five calls take the mean-field input to quasiparticle energies:
 *
 *   gw_build_gt       imaginary-time density matrices            (Eq. 2)
 *   gw_contract_chi   block-sparse polarizability chi_PQ(i tau)  (Eq. 3)
 *   gw_screen_w       chi(i w), epsilon, W^c(i w), W^c(i tau)    (Eqs. 5-9)
 *   gw_contract_sigma diagonal Sigma^c_n(i tau) and Sigma^x_n    (Eqs. 10-11)
 *   gw_continue_qp    transforms, Pade, Newton on the QP eq.     (Eq. 12)
 *
 * Real convention used throughout (the printed i-factors of Eqs. 2, 3, 10
 * dropped; same physics): energies are shifted by mu_F,
 *   D^occ(tau) = sum_{i occ} exp(+(eps_i - mu_F) tau) c_i c_i^T
 *   D^vir(tau) = sum_{a vir} exp(-(eps_a - mu_F) tau) c_a c_a^T,  tau >= 0
 *   chi_PQ(tau) = - sum_{mu sigma} [sum_l (l sigma P) D^occ_{mu l}]
 *                                  [sum_nu (mu nu Q) D^vir_{nu sigma}]
 * (per spin channel; negative semidefinite).
 *
 * Conventions of every call:
 *  - Pointers marked "dev" are device pointers, "host" are host pointers.
 *  - The caller owns and allocates inputs and outputs; the library never
 *    frees caller memory.  Calls allocate and free their own scratch
 *    (stream-ordered) and return GW_ERR_NOMEM when that fails.
 *  - Calls are asynchronous on `stream` except where a result is written to
 *    host memory (then they synchronize the stream before returning).
 *  - Arguments are validated on the host before any launch; on error nothing
 *    is launched and gw_last_error() describes the problem.
 *  - Matrices are row-major FP64.  Atoms carry ao_per_atom AO and
 *    ri_per_atom RI functions, or per-atom counts given by offsets (gw_system).
 */
#ifndef GW_H_
#define GW_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gw_status;
enum {
  GW_OK = 0,
  GW_ERR_ARG = 1,          /* invalid argument (nothing launched)            */
  GW_ERR_HIP = 2,          /* a HIP runtime call failed                      */
  GW_ERR_NOMEM = 3,        /* scratch allocation failed                      */
  GW_ERR_NOT_SPD = 4,      /* Cholesky of V or of epsilon(i w) failed        */
  GW_ERR_NO_CONVERGE = 5,  /* Newton did not converge for at least one state */
  GW_ERR_BLAS = 6,         /* rocBLAS / rocSOLVER returned an error          */
  GW_ERR_AUDIT = 7         /* the screener skipped an output block that the
                              exact contraction keeps (gw_contract_chi audit) */
};

/* Arithmetic of the chi contraction: GW_FP64 (FP64 MFMA throughout),
 * GW_FP32 (operands and half-contracted tensors rounded to FP32, FP32 MFMA
 * products with FP32 accumulation inside a tile, FP64 accumulation of chi
 * across pivots) or GW_BF16X3 (operands split into bf16 hi + lo, three bf16
 * MFMA products with FP32 accumulation inside a tile, FP64 accumulation
 * across pivots; ao_per_atom <= 16, else GW_ERR_ARG). */
typedef enum { GW_FP64 = 0, GW_FP32 = 1, GW_BF16X3 = 2 } gw_prec;

/* One molecule / strip.  Atom-triple bricks (a, b, c) of the three-center
 * tensor (mu nu|P) (Eq. 4): mu on AO atom a, nu on AO atom b, P on RI atom c.
 * Brick i of `trip` is stored at t3c + i * ao_per_atom^2 * ri_per_atom as
 * [mu][nu][P] row-major.  The list must contain (b, a, c) whenever it contains
 * (a, b, c) (the tensor is symmetric in mu nu); triples left out are zero.
 *
 * Atoms of different elements (the paper's nanoribbons: C and H) carry
 * different numbers of functions: ao_off / ri_off then give atom a the
 * functions ao_off[a] .. ao_off[a+1]-1 (1 .. ao_per_atom of them) and
 * ri_off[a] .. ri_off[a+1]-1 (1 .. ri_per_atom); n_ao = ao_off[n_atoms],
 * n_ri = ri_off[n_atoms], and every matrix argument (C, D, chi, V, W, S) has
 * these compact sizes.  The bricks keep the per-atom maxima: element
 * (mu, nu, P) of brick (a, b, c) for the function numbers mu, nu, P within
 * the atoms, zero where a function does not exist.  The calls with atom-block
 * structure (gw_contract_chi, gw_contract_sigma) run on the padded form (the
 * missing functions as zero functions) and convert their inputs and outputs;
 * the flop counts in their statistics are those of the padded blocks.  The
 * batched plans, the block screener and gw_t3c_gaussian take systems without
 * offsets only (GW_ERR_ARG). */
typedef struct {
  int32_t n_atoms;
  int32_t ao_per_atom;     /* n_ao = n_atoms * ao_per_atom (without ao_off)  */
  int32_t ri_per_atom;     /* n_ri = n_atoms * ri_per_atom (without ri_off)  */
  int32_t n_occ;           /* occupied MOs, 1 <= n_occ < n_ao                */
  int64_t n_trip;
  const int32_t *trip;     /* host [n_trip][3] = (a, b, c)                   */
  const double *t3c;       /* dev  [n_trip][ao][ao][ri]                      */
  const double *xyz;       /* host [n_atoms][3] bohr, or NULL; only the block
                              screener uses it (distance feature) and then
                              requires it                                     */
  const int32_t *ao_off;   /* host [n_atoms+1] per-atom AO offsets, or NULL  */
  const int32_t *ri_off;   /* host [n_atoms+1] per-atom RI offsets, or NULL  */
} gw_system;

/* Block screener network (beyond the paper): a perceptron x (F) -> 64 -> 64
 * -> 1 with ReLU, predicting log10 of the Frobenius norm of a chi output atom
 * block (c, c', tau).  Parameters packed [w1 64*F][b1 64][w2 64*64][b2 64]
 * [w3 64][b3 1] (gw_mlp_param_count floats).  All buffers are caller-owned
 * device arrays; `step` is the Adam step counter (updated by the library). */
typedef struct {
  int32_t n_features;      /* F, 1..16 (gw_chi_block_features writes 6)      */
  int32_t hidden;          /* must be 64                                      */
  int32_t step;
  float *params;           /* dev FP32 master parameters                     */
  void *params16;          /* dev FP16 copy used for inference               */
  float *adam_m, *adam_v;  /* dev Adam moments                               */
  float *grad;             /* dev gradient buffer                            */
} gw_mlp;

/* Imaginary-time density matrices (Eq. 2).
 * C: dev [n_ao][n_ao], row n = MO n (orthonormal AO basis); eps: host [n_ao],
 * the first n_occ occupied, each occupied level below mu_f and each virtual
 * level above it (in any order otherwise: an evGW update may reorder levels);
 * tau: host [n_tau] >= 0.  Writes d_occ, d_vir: dev [n_tau][n_ao][n_ao].
 * Either output may be NULL to skip it.
 * Errors: GW_ERR_ARG for bad sizes, non-finite eps, occupied (virtual) levels
 * not below (above) mu_f, negative/non-finite tau. */
gw_status gw_build_gt(const gw_system *s, const double *C, const double *eps, double mu_f,
                      int32_t n_tau, const double *tau, double *d_occ, double *d_vir,
                      hipStream_t stream);

/* gw_build_gt without any allocation, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc): the per-tau weights are staged in an array the
 * library holds on every device it runs on (8 MiB, kept until the process
 * ends) instead of call-owned scratch.  Arguments, layouts, outputs and
 * errors as gw_build_gt, plus GW_ERR_ARG when 2 * n_tau * n_ao exceeds
 * 2^20 (the array's size in doubles).  Every call on one device shares that
 * device's array: calls that overlap on one device (different streams, or
 * host threads) race and must be ordered by the caller. */
gw_status gw_build_gt_noalloc(const gw_system *s, const double *C, const double *eps,
                              double mu_f, int32_t n_tau, const double *tau, double *d_occ,
                              double *d_vir, hipStream_t stream);

typedef struct {
  int32_t prec;            /* gw_prec                                         */
  double filter_eps;       /* atom-block filter (Frobenius norm), >= 0        */
  int32_t timing;          /* 1: time every stage launch with HIP events on
                              `stream` (fills ms_stage)                        */
  const gw_mlp *screener;  /* NULL, or a trained block screener: output blocks
                              (c, c', tau) predicted below
                              log10(filter_eps) - screen_margin are neither
                              computed nor kept (zero); needs filter_eps > 0   */
  double screen_margin;    /* decades of safety band below the filter          */
  const double *screen_tau;/* host [n_tau] tau values (screener feature)       */
  int32_t keep_small_blocks; /* 1: skip the output filter (chi blocks below
                              filter_eps are kept; for audits of the skipped
                              mass); 0: the filter of the computational details */
  int32_t screen_audit;    /* with a screener: 1 = judge the skipped blocks by
                              the exact contraction (the same call run again
                              without the screener, on call-owned scratch of
                              one chi stack): a skipped block whose exact norm
                              is >= filter_eps (one the filter keeps) fails
                              the audit                                        */
  int32_t screen_fallback; /* with screen_audit: 1 = on a failed audit return
                              the exact chi (bit-equal to the call without a
                              screener) and GW_OK; 0 = return GW_ERR_AUDIT with
                              the screened chi left in `chi`                    */
} gw_chi_opts;

typedef struct {
  int64_t n_trip_kept;     /* bricks at or above the filter                   */
  int64_t n_dblk_dropped;  /* D(tau) atom blocks below the filter (all tau)   */
  int64_t n_chiblk_dropped;/* chi output atom blocks zeroed (all tau)         */
  double flops_ab;         /* algorithmic flops of the two half contractions  */
  double flops_c;          /* algorithmic flops of the outer contraction      */
  double ms_total;         /* wall time of the call (host clock, synchronized)*/
  double ms_stage[3];      /* summed kernel time of the half contractions A,
                              B and of the outer contraction C (timing = 1)   */
  int64_t n_launch[3];     /* launches of each stage                          */
  double flops_stage[3];   /* algorithmic flops of each stage                 */
  int64_t n_blocks_screened; /* (c <= c', tau) output blocks the screener skipped */
  int64_t n_tiles_screened;  /* outer-contraction tiles skipped by the screener */
  int32_t c_variant;       /* stage-C tile variant used (see gw_chi_batch_*)    */
  int32_t launch_mask;     /* stages launched in the persistent form (bit k)    */
  int32_t audit_done;      /* 1 when the screener audit ran                    */
  int32_t audit_fallback;  /* 1 when the audit failed and the exact chi was
                              returned (screen_fallback)                       */
  int64_t n_audit_violations; /* skipped blocks the exact filter keeps        */
  double audit_max_skipped;/* largest exact Frobenius norm of a skipped block */
  double audit_skipped_mass; /* sqrt(sum of squared exact norms of the skipped
                              blocks) / Frobenius norm of the exact chi        */
  double audit_ms;         /* wall time of the audit (host clock)             */
} gw_chi_stats;

/* Three-center overlap integrals (Eq. 4), (mu nu P) = int phi_mu phi_nu phi_P dr,
 * of s-type Gaussian basis functions, written as the system's bricks.  Every
 * atom carries the same functions: AO function i at xyz[atom] + ao_offset[i]
 * with exponent ao_exp[i] (i < ao_per_atom), RI function p at xyz[atom] +
 * ri_offset[p] with exponent ri_exp[p], each normalized,
 * g(r) = (2a/pi)^(3/4) exp(-a |r - R|^2); by the Gaussian product theorem
 *   (mu nu P) = N_a N_b N_c (pi/s)^(3/2) exp(-(ab|A-B|^2 + ac|A-C|^2 + bc|B-C|^2)/s),
 * s = a + b + c.  s: n_atoms, sizes, the triple list (host) and xyz (host,
 * bohr) are read; s->t3c is ignored.  ao_exp host [ao_per_atom], ri_exp host
 * [ri_per_atom] (> 0); ao_offset host [ao_per_atom][3], ri_offset host
 * [ri_per_atom][3] (bohr), either may be NULL for functions at the atoms.
 * t3c: dev [n_trip][ao][ao][ri], overwritten (the brick layout of gw_system).
 * Asynchronous on stream.  Errors: GW_ERR_ARG (sizes, null or non-finite
 * inputs, exponents <= 0), GW_ERR_NOMEM, GW_ERR_HIP. */
gw_status gw_t3c_gaussian(const gw_system *s, const double *ao_exp, const double *ao_offset,
                          const double *ri_exp, const double *ri_offset, double *t3c,
                          hipStream_t stream);

/* Polarizability chi_PQ(tau_j) for all tau at once (Eq. 3), with the atom-block
 * filter of the paper's computational details: bricks of norm < filter_eps and
 * D(tau) atom blocks of norm < filter_eps are dropped, then chi atom blocks of
 * norm < filter_eps are zeroed.
 * d_occ, d_vir: dev [n_tau][n_ao][n_ao] (symmetric); chi: dev
 * [n_tau][n_ri][n_ri], overwritten, symmetric (upper blocks computed,
 * mirrored).  stats (host, may be NULL) is filled.  The call is synchronous:
 * it reads the kept-brick mask on the host first and releases its scratch
 * (plain device allocations) before returning.  It runs the batched form
 * below on one system, eagerly, with the default tile configuration of the
 * precision (the fastest measured on gfx950 for 13 AO / 40 RI per atom:
 * FP64 stage-C variant 3 (the direct-to-LDS outer contraction; variant 2
 * when ri_per_atom is odd) with all stages persistent, FP32 variant 3
 * (variant 0 when ri_per_atom is not a multiple of 4) with stages B and C
 * persistent (stage B as a grid when the
 * basis has at most 64 AO x RI functions per atom pair), BF16x3 variant 3
 * (its direct-to-LDS outer contraction) with all stages persistent).
 * With a block screener (opts->screener, beyond the paper; the filter idea of
 * the computational details) the output blocks (c <= c', tau) predicted below
 * log10(filter_eps) - screen_margin are not computed and left zero (the
 * outer-contraction tiles, the half-contracted N_b column blocks and M_b row
 * tiles that only such blocks use are skipped); blocks in the band above that
 * are computed exactly.  opts->screen_audit makes the
 * exact contraction the judge: the call runs again without the screener and
 * every skipped block is compared with the filter's decision on the exact
 * result (stats: violations, largest skipped norm, skipped mass).  A failed
 * audit returns GW_ERR_AUDIT, or with opts->screen_fallback the exact chi.
 * Errors: GW_ERR_ARG (sizes, pointers, options), GW_ERR_NOMEM, GW_ERR_HIP,
 * GW_ERR_AUDIT. */
gw_status gw_contract_chi(const gw_system *s, const double *d_occ, const double *d_vir,
                          int32_t n_tau, const gw_chi_opts *opts, double *chi,
                          gw_chi_stats *stats, hipStream_t stream);

/* Batched persistent form of gw_contract_chi (Eq. 3 for many independent
 * systems, e.g. the molecules of a benchmark set).
 *
 * A plan is made once per set of systems: it filters and groups the bricks
 * of every system (brick norms are read on the host), lays out the stage-C
 * column panels, allocates the scratch of one pivot's half-contracted
 * tensors per system (plain device allocations, held until destroy) and,
 * for GW_BF16X3, splits the bricks into bf16 hi/lo once.  The plan is valid
 * for the brick VALUES present at creation: t3c pointers and contents must
 * not change until gw_chi_batch_destroy.  All systems must share
 * ao_per_atom and ri_per_atom; opts->screener must be NULL.
 *
 * An execution walks the pivot atom index i = 0 .. max n_atoms - 1 and
 * issues, per stage, one launch over the tiles of every system with a pivot
 * atom i, for all n_tau points at once.  Stage B (the D^vir half
 * contraction) runs once per group of consecutive pivots (up to 128 rows of
 * pivot x tau x function per tile in FP64, 160 otherwise).  A system whose
 * pivot atoms i and i + ceil(n_atoms/2) never couple to a common RI atom
 * runs them in the same launches (their chi rows are disjoint; the second
 * pivot's half-contracted tensors take a second set of buffers, if within
 * 32 GiB): the loop then has ceil(n_atoms/2) steps.  Results equal n_sys
 * calls of gw_contract_chi with the same opts (same arithmetic, same order
 * of every sum).
 *
 * gw_chi_batch_create: systems host [n_sys]; *plan receives the handle.
 *   Synchronizes `stream`.
 * gw_chi_batch_execute: d_occ, d_vir, chi are HOST arrays of n_sys device
 *   pointers with the layouts of gw_contract_chi (chi overwritten).
 *   use_graph = 0: eager launches (opts->timing fills ms_stage);
 *   use_graph = 1: the launch sequence is captured into a hipGraph on first
 *   use and replayed afterwards; it is captured again when any pointer, the
 *   stream or the tile configuration changes.  Needs a created (non-NULL)
 *   stream.  Without stats the call is asynchronous; with stats it
 *   synchronizes to read the filter counts.  Calls on one plan must not
 *   overlap (they share its scratch).
 * gw_chi_batch_set_config / get_config: stage-C tile variant
 *   (0 .. n_variants-1) and launch modes: persistent is a mask, bit k set =
 *   stage k (0: A, 1: B, 2: C) runs as a resident grid that takes tiles from
 *   per-XCD device queues, largest systems first; bit clear = one workgroup
 *   per tile (XCD-aware tile order).  ARG error outside these ranges, and
 *   for variant 3 of FP64 / FP32 plans when ri_per_atom is not a multiple of
 *   2 / 4 (its operands are copied into LDS 16 bytes at a time).
 * gw_chi_batch_tune: autotuner.  If cache_path (may be NULL) holds an entry
 *   for the plan's shape class (precision, AO/RI per atom, n_tau, log2 of
 *   the system count and of the mean atom count) that configuration is
 *   taken; otherwise every usable variant is run in both launch modes (reps timed
 *   executions each, stage times from HIP events), each stage takes its
 *   fastest mode and stage C its fastest variant, and the result is
 *   appended to cache_path.  *ms_out (host, may be NULL) receives the time
 *   per execution of the chosen configuration.  Overwrites chi.
 * gw_chi_batch_destroy: releases the plan (synchronizes the device). */
typedef struct gw_chi_batch gw_chi_batch;

gw_status gw_chi_batch_create(int32_t n_sys, const gw_system *systems, int32_t n_tau,
                              const gw_chi_opts *opts, gw_chi_batch **plan, hipStream_t stream);
gw_status gw_chi_batch_execute(gw_chi_batch *plan, const double *const *d_occ,
                               const double *const *d_vir, double *const *chi,
                               int32_t use_graph, gw_chi_stats *stats, hipStream_t stream);
gw_status gw_chi_batch_set_config(gw_chi_batch *plan, int32_t variant, int32_t persistent);
/* gw_chi_batch_set_engine: engine of the half contractions (stages A and B):
 *   0 (default): the direct-to-LDS engine wherever the plan's rows allow its
 *   16-byte copies, else the register-staged one; 1: the register-staged
 *   engine.  Both take the same k values in the same order into every sum:
 *   the results are bit-identical.  A captured graph is dropped.  ARG error
 *   for other values. */
gw_status gw_chi_batch_set_engine(gw_chi_batch *plan, int32_t engine);
gw_status gw_chi_batch_get_config(const gw_chi_batch *plan, int32_t *variant,
                                  int32_t *persistent, int32_t *n_variants);
gw_status gw_chi_batch_tune(gw_chi_batch *plan, const double *const *d_occ,
                            const double *const *d_vir, double *const *chi, int32_t reps,
                            const char *cache_path, double *ms_out, hipStream_t stream);
gw_status gw_chi_batch_destroy(gw_chi_batch *plan);

/* Screening (Eqs. 5-9) with RI overlap metric S = 1:
 *   chi(i w_k) = 2 spin sum_j cos_w[k][j] chi(tau_j)
 *   V = L L^T, eps(i w_k) = 1 - L^T chi(i w_k) L
 *   W^c(i w_k) = L [eps^-1 - 1] L^T
 *   wc(tau_j)  = 1/2 sum_k icos_w[j][k] W^c(i w_k)
 * chi: dev [n_tau][n_ri][n_ri]; V: dev [n_ri][n_ri] SPD; cos_w: host
 * [n_w][n_tau]; icos_w: host [n_tau][n_w]; wc: dev [n_tau][n_ri][n_ri].
 * Errors: GW_ERR_NOT_SPD when V or some eps(i w_k) is not positive definite
 * (the stream is synchronized to read the factorization status). */
gw_status gw_screen_w(const gw_system *s, const double *chi, const double *V, int32_t n_tau,
                      int32_t n_w, const double *cos_w, const double *icos_w, double spin,
                      double *wc, hipStream_t stream);
/* Open-shell (spin-polarized) screening: gw_screen_w with chi = chi_up +
 * chi_dn and spin factor 1.  chi_up, chi_dn: dev [n_tau][n_ri][n_ri], the
 * per-channel polarizabilities of gw_contract_chi (two systems sharing the
 * bricks, each with its channel's n_occ, the Green's functions built with one
 * common mu_F); read only, caller-owned.  The sum is taken inside the cosine
 * transform; nothing else differs from gw_screen_w (same workspace, errors
 * and stream semantics), plus GW_ERR_ARG for a null chi_up or chi_dn.  The
 * paper writes Eqs. 5-9 for a closed shell and runs its nanoribbons as
 * open-shell singlets (computational details): two channels, one W. */
gw_status gw_screen_w_spins(const gw_system *s, const double *chi_up, const double *chi_dn,
                            const double *V, int32_t n_tau, int32_t n_w, const double *cos_w,
                            const double *icos_w, double *wc, hipStream_t stream);
/* Screening with a non-orthogonal RI basis (Eq. 5 and the definitions after
 * Eqs. 10 and 11): with the RI overlap S_PQ the dielectric function takes
 * chi~ = S^-1 chi S^-1, and the self-energies take W~^c = S^-1 W^c S^-1 and
 * V~ = S^-1 V S^-1.  S_ri: dev [n_ri][n_ri], symmetric positive definite,
 * read only, caller-owned.  wc_tilde: dev [n_tau][n_ri][n_ri], overwritten
 * with W~^c(tau_j), to be passed to gw_contract_sigma as its wc; v_tilde: dev
 * [n_ri][n_ri] or NULL, overwritten with V~, to be passed to
 * gw_contract_sigma as its V.  Other arguments, workspace and stream
 * semantics as gw_screen_w; no output may alias an input.  Errors as
 * gw_screen_w, plus GW_ERR_ARG for a null S_ri and GW_ERR_NOT_SPD when S is
 * not positive definite.  S_ri = 1 gives gw_screen_w's W^c (and V~ = V). */
gw_status gw_screen_w_metric(const gw_system *s, const double *chi, const double *V,
                             const double *S_ri, int32_t n_tau, int32_t n_w, const double *cos_w,
                             const double *icos_w, double spin, double *wc_tilde,
                             double *v_tilde, hipStream_t stream);
/* Both at once, as the paper's open-shell ribbons need (overlap-metric RI,
 * two spin channels): gw_screen_w_metric of chi = chi_up + chi_dn with spin
 * factor 1 (chi_up, chi_dn as for gw_screen_w_spins).  Outputs, errors and
 * stream semantics as gw_screen_w_metric. */
gw_status gw_screen_w_spins_metric(const gw_system *s, const double *chi_up,
                                   const double *chi_dn, const double *V, const double *S_ri,
                                   int32_t n_tau, int32_t n_w, const double *cos_w,
                                   const double *icos_w, double *wc_tilde, double *v_tilde,
                                   hipStream_t stream);

/* Coulomb matrix of a periodic Gamma-point cell (Eq. 8; the paper obtains V
 * for periodic cells by Ewald summation).  The RI functions are normalized
 * Gaussian charges: centres host [n_ri][3] (bohr), alpha host [n_ri] (> 0),
 * in the orthorhombic cell with box lengths cell host [3] (bohr), with a
 * neutralizing background (G = 0 left out):
 *   V_PQ = (4 pi/Omega) sum_{G != 0} e^{-G^2/4a_P} e^{-G^2/4a_Q} cos(G.(R_P - R_Q)) / G^2.
 * Computed by an Ewald split with parameter eta (0: chosen by a cost model;
 * else 0 < eta < sqrt(min alpha / 2)): a real-space erf sum over lattice
 * images, a reciprocal sum as one FP64 GEMM, and the background constant;
 * terms below tol (0 < tol <= 1e-6; 1e-17 for full FP64) are dropped.  V:
 * dev [n_ri][n_ri], overwritten (symmetric).  info: host, optional (NULL),
 * receives the parameters used.  Synchronous on stream; the workspace
 * (n_ri x 2 n_g doubles) is allocated stream-ordered and freed.  Errors:
 * GW_ERR_ARG for bad sizes, pointers, exponents, cell, tol or eta, or a
 * split whose image box or reciprocal list exceeds the bounds; GW_ERR_NOMEM,
 * GW_ERR_BLAS, GW_ERR_HIP. */
typedef struct {
  double eta;     /* splitting parameter used                          */
  double r_cut;   /* real-space cutoff (bohr)                           */
  double g_cut;   /* reciprocal cutoff (1/bohr)                         */
  int32_t n_g;    /* reciprocal vectors in the half space               */
  int32_t n_img;  /* lattice images each element of V visits            */
} gw_coulomb_info;
gw_status gw_coulomb_periodic(int32_t n_ri, const double *centres, const double *alpha,
                              const double *cell, double eta, double tol, double *V,
                              gw_coulomb_info *info, hipStream_t stream);

typedef struct {
  double flops;            /* algorithmic flops of the self-energy products   */
  double ms_total;
} gw_sigma_stats;

/* Diagonal self-energy pieces (Eqs. 10-11) for the listed MOs:
 *   B^n_{mu P}      = sum_nu C_{n nu} (nu mu P)
 *   sig_occ[n][j]   = <D^occ(tau_j), B^n W^c(tau_j) B^nT>_F
 *   sig_vir[n][j]   = <D^vir(tau_j), B^n W^c(tau_j) B^nT>_F
 *   sig_x[n]        = -<D^occ(0), B^n V B^nT>_F
 * The same filter as gw_contract_chi is applied to the bricks and to the D
 * atom blocks.  states: host [n_gw] MO indices; C: dev [n_ao][n_ao];
 * d_occ, d_vir, wc: dev stacks of n_tau; d_occ0: dev [n_ao][n_ao] = D^occ(0);
 * V: dev [n_ri][n_ri]; outputs are host arrays (the call synchronizes).
 * d_occ0, V and sig_x may all be NULL together: the exchange term (which does
 * not depend on tau) is then skipped, e.g. when the tau points are contracted
 * one call at a time; giving only some of the three is GW_ERR_ARG. */
gw_status gw_contract_sigma(const gw_system *s, int32_t n_gw, const int32_t *states,
                            const double *C, const double *d_occ, const double *d_vir,
                            const double *d_occ0, const double *wc, const double *V,
                            int32_t n_tau, double filter_eps, double *sig_occ, double *sig_vir,
                            double *sig_x, gw_sigma_stats *stats, hipStream_t stream);
/* The same with the precision of the per-slot products (the bulk of
 * Eq. 10-11): GW_FP64 (= gw_contract_sigma) or GW_FP32 (precision form:
 * W^c(tau_j), V and B^n rounded to FP32, FP32 products and tile sums, the
 * tile dots with D summed in FP64; the half transform to B^n stays FP64).
 * ARG error for GW_BF16X3. */
gw_status gw_contract_sigma_prec(const gw_system *s, int32_t n_gw, const int32_t *states,
                                 const double *C, const double *d_occ, const double *d_vir,
                                 const double *d_occ0, const double *wc, const double *V,
                                 int32_t n_tau, double filter_eps, int32_t prec, double *sig_occ,
                                 double *sig_vir, double *sig_x, gw_sigma_stats *stats,
                                 hipStream_t stream);

typedef struct {
  double pade_window;      /* use only nodes with w_k <= window (Ha); <= 0:
                              all; GW_PADE_WINDOW_HA is the paper's 10 eV     */
  double newton_tol;       /* stop when |dE| < tol (Ha); <= 0: 1e-10           */
  int32_t max_iter;        /* <= 0: 100                                        */
} gw_qp_opts;

/* The analytic continuation window of the paper's computational details,
 * i[0, +10 eV] for virtual and i[0, -10 eV] for occupied states, in hartree
 * (CODATA 2018: 1 Ha = 27.211386245988 eV). */
#define GW_PADE_WINDOW_HA (10.0 / 27.211386245988)

/* Quasiparticle energies (Eq. 12), host only:
 *   Sigma^c_n(i w_k) = sum_j cos_w[k][j] (vir - occ)[n][j]
 *                      + i sum_j sin_w[k][j] (vir + occ)[n][j]
 * Thiele continued-fraction Pade on nodes +i w_k (virtual states) or -i w_k
 * with conjugated values (occupied), w_k <= opts->pade_window (opts NULL:
 * GW_PADE_WINDOW_HA, newton_tol 1e-10, 100 iterations), then Newton from
 * E = eps_n on
 *   E - eps_n + vxc_n - sig_x_n - Re Sigma^c_n(E - mu_F) = 0.
 * state_status[n] = GW_OK or GW_ERR_NO_CONVERGE (e_qp[n] = NaN then); the
 * call returns GW_ERR_NO_CONVERGE if any state failed. */
gw_status gw_continue_qp(int32_t n_gw, const double *sig_occ, const double *sig_vir,
                         const double *sig_x, const double *eps_n, const double *vxc_n,
                         const int32_t *is_occ, double mu_f, int32_t n_tau, int32_t n_w,
                         const double *omega, const double *cos_w, const double *sin_w,
                         const gw_qp_opts *opts, double *e_qp, int32_t *state_status);

/* Eigenvalue self-consistent GW (evGW; the paper's step after Eq. 12: the QP
 * energies replace the mean-field levels in the Green's function, Eq. 2, and
 * the cycle repeats until they are self-consistent), host only: the energies
 * of the next Green's function.  eps0: [n_mo] mean-field energies, the first
 * n_occ occupied; states / e_qp: [n_gw] computed states (distinct, in
 * [0, n_mo)) and their QP energies.  eps_out[i] (host [n_mo]) = e_qp of state
 * i if computed, else eps0[i] + the mean correction e_qp - eps0 of the computed
 * states of its class (occupied i < n_occ, virtual otherwise; no shift for a
 * class without computed states).  *mu_out = midpoint of the highest occupied
 * and the lowest virtual eps_out.  The QP equation of the next cycle keeps
 * eps0 and v^xc.  ARG error for invalid arguments or non-finite e_qp;
 * GW_ERR_NO_CONVERGE (eps_out and *mu_out filled) when an occupied level ends
 * at or above a virtual one: the Green's function of Eq. 2 would not decay. */
gw_status gw_evgw_update(int32_t n_mo, int32_t n_occ, const double *eps0, int32_t n_gw,
                         const int32_t *states, const double *e_qp, double *eps_out,
                         double *mu_out);

/* Energy zero mu_F of the Green's function (Eq. 2 decays with tau only for
 * occupied levels below mu_F and virtual levels above it), host only: the
 * midpoint of the highest occupied and the lowest virtual level over n_chan
 * channels (1: closed shell; 2: the spin channels of an open shell, which
 * share one mu_F).  n_mo, n_occ: host [n_chan]; eps: host [n_chan] arrays of
 * n_mo[c] energies, the first n_occ[c] occupied.  *mu_out receives mu_F.
 * GW_ERR_ARG for bad arguments, non-finite energies, or an occupied level at
 * or above a virtual level of any channel. */
gw_status gw_fermi_level(int32_t n_chan, const int32_t *n_mo, const int32_t *n_occ,
                         const double *const *eps, double *mu_out);

/* Screener features of every output block: dev [n_tau][n_atoms][n_atoms][6] =
 * (distance/10 bohr, log10 tau, log10 ||T_c||, log10 ||T_c'||,
 *  log10 ||D^occ_{cc'}(tau)||, log10 ||D^vir_{cc'}(tau)||) with norms over the
 * kept bricks of RI atom c and over the (c, c') atom blocks of D (1e-30 added
 * inside every log).  tau: host [n_tau].  s->xyz must be set (GW_ERR_ARG
 * otherwise: without it the distance feature would be zero). */
gw_status gw_chi_block_features(const gw_system *s, const double *d_occ, const double *d_vir,
                                int32_t n_tau, const double *tau, double filter_eps, float *feat,
                                hipStream_t stream);
/* log10(||chi_{cc'}(tau)|| + 1e-30) of every RI atom block: dev [n_tau][na][na]. */
gw_status gw_chi_block_lognorms(const gw_system *s, const double *chi, int32_t n_tau,
                                float *out, hipStream_t stream);

/* Screener network calls (training and inference run on the GPU): */
int64_t gw_mlp_param_count(int32_t n_features, int32_t hidden);   /* -1 if unsupported */
/* y[n] = net(x[n][F]); use_fp16 selects the FP16 copy of the weights. */
gw_status gw_mlp_forward(const gw_mlp *net, int64_t n, const float *x, float *y,
                         int32_t use_fp16, hipStream_t stream);
/* Gradient of the asymmetric loss mean(w(r) r^2), r = net(x) - t, w = 1 for
 * r >= 0 and alpha for r < 0, into grad (dev [P]); loss into loss_dev (dev). */
gw_status gw_mlp_gradient(const gw_mlp *net, int32_t n, const float *x, const float *t,
                          float alpha, float *grad, float *loss_dev, hipStream_t stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on a batch; refreshes params16. */
gw_status gw_mlp_train_step(gw_mlp *net, int32_t n, const float *x, const float *t, float alpha,
                            float lr, float *loss_dev, hipStream_t stream);
/* params16 <- params (after the caller changed the FP32 parameters). */
gw_status gw_mlp_sync_half(gw_mlp *net, hipStream_t stream);

/* Releases the state the library keeps between calls outside plans (the
 * per-device rocBLAS / rocSOLVER handles of the screening calls); plans are
 * released by gw_chi_batch_destroy.  Later calls recreate the state on
 * demand.  Must not overlap with other calls into the library. */
gw_status gw_finalize(void);

/* Message of the last failing call on this thread ("" if none). */
const char *gw_last_error(void);
/* Library version string. */
const char *gw_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GW_H_ */
