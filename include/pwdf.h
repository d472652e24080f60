/*
 * pwdf.h -- C ABI of libpwdf: the long-range (reciprocal-space) Coulomb matrix
 * of a periodic Gaussian basis by integral-direct planewave density fitting,
 * on AMD Instinct MI355X (gfx950).
 *
 * Method: Dinh, Rettig, Feng, Lee, "Efficient All-Electron Periodic
 * Fourier-Transformed Coulomb Method", arXiv 2509.16460, section "Long-range
 * contributions" (eq. "AFT for pair density" and the three-step contraction
 * order that follows it), eq. "Ewald J" (second term), eq. "FT for D" and
 * eq. "FT of J".  For every screened primitive pair (a in cell 0, b in cell L)
 * the analytic Fourier transform F_abL(G) of the Gaussian product is formed on
 * the fly and contracted with the real-space density:
 *
 *   D(L)     = sum_k w_k e^{ik.L} D(k)                       (w_k = 1/Nk)
 *   rho(G)   = (1/Omega) sum_{(a,b,L)} D_ab(L) F_abL(G)
 *   v(G)     = 4 pi exp(-|G|^2 / 4 omega^2) / |G|^2,  G != 0
 *   J_ab(L)  = sum_G v(G) rho(-G) F_abL(G)
 *   J(k)     = sum_L e^{ik.L} J(L)
 *   E_J      = 1/2 Omega sum_G v(G) |rho(G)|^2 = 1/2 sum_k w_k sum D(k) J(k)
 *
 * G runs over {G = B n : 0 < |G| <= 2 omega sqrt(-ln eps_G)}, B = 2 pi A^-T
 * (appendix "Cartesian coordinates and relative coordinates"); pairs are kept
 * when the Gaussian-product prefactor exp(-a_a a_b/(a_a+a_b) |A-B-L|^2) is at
 * least eps_pair (and |A-B-L| <= r_max when r_max > 0).
 *
 * Conventions
 *   lattice   3x3 row-major, rows a1, a2, a3 (Bohr).  Omega = |det|.
 *   basis     Cartesian shells, l <= 3; components in descending lexicographic
 *             (lx,ly,lz) order; each primitive carries
 *             N(l,a) = (2a/pi)^{3/4} (4a)^{l/2} / sqrt((2l-1)!!) times its
 *             contraction coefficient.  nbf = sum over shells of (l+1)(l+2)/2.
 *   k-mesh    Gamma-centred: k = sum_i (m_i/n_i) b_i, m_i = 0..n_i-1, index
 *             (m1*n2 + m2)*n3 + m3.
 *   D(k),J(k) complex128 interleaved (re, im), [ndm][nk][nbf][nbf] row-major;
 *             D(L) pairs phi_mu in cell 0 with phi_nu in cell L.  Each D(k)
 *             must be Hermitian: of each pair D_mu,nu(k), D_nu,mu(k) only one
 *             is read (chosen per shell pair), so a non-Hermitian input gives
 *             a mix of its two triangles.  J(k) is Hermitian.
 *
 * Ownership and streams
 *   The caller owns every input and output buffer; the library never frees or
 *   retains them.  The library owns the context (plan and device workspaces),
 *   allocated in pwdf_create; pwdf_build_j and pwdf_grad do not allocate.
 *   Device calls only enqueue work on the given HIP stream (NULL: the null
 *   stream); results are valid after the stream is synchronised.  Independent
 *   launches inside one call (the class groups of a pass) either fan out over
 *   internal streams of the context (default priority) and join back into the
 *   given stream before the next dependent step, or follow each other on it
 *   (pwdf_stats.fork, chosen by pwdf_autotune; default: fan out); stream order
 *   is preserved either way.  One context must not be
 *   used by two streams at once: calls on one context that overlap in time
 *   (different streams, or a graph replay racing an eager call) race on its
 *   workspaces.  Distinct contexts are independent.
 *
 * Errors
 *   Every call returns a pwdf_status; nothing aborts.  Arguments are validated
 *   on the host before anything is enqueued; on failure nothing is enqueued and
 *   pwdf_last_error(ctx) describes the problem (pwdf_last_error(NULL) reports
 *   the last failure of the calling thread that had no context: a failed
 *   pwdf_create, or a call given a NULL ctx).  HIP runtime failures map to
 *   PWDF_EDEVICE with the HIP error string (PWDF_ENOMEM for an allocation).
 */
#ifndef PWDF_H
#define PWDF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pwdf_ctx pwdf_ctx;

typedef enum {
  PWDF_OK = 0,
  PWDF_EINVAL = -1,       /* bad argument, shape or geometry */
  PWDF_ENOMEM = -2,       /* host or device allocation failed */
  PWDF_EDEVICE = -3,      /* HIP runtime error */
  PWDF_EUNSUPPORTED = -4, /* l > 3, ndm > max_ndm, unsupported precision */
  PWDF_ENONFINITE = -5,   /* non-finite input */
  PWDF_ESTATE = -6        /* call out of order (e.g. gradient before any plan) */
} pwdf_status;

typedef enum {
  PWDF_FP64 = 0,      /* every step in FP64 */
  PWDF_FP32_MFMA = 1  /* pair-G tiles generated in FP32, contracted on FP32 MFMA,
                         FP64 accumulation across pairs; phase sums, E-coefficient
                         transforms and the energy stay FP64.  The head of the G
                         set -- the G whose Coulomb weight v(G) is at least 2^-20
                         of the largest (pwdf_set_fp32_head), a ball around G = 0
                         -- takes FP64 tiles on FP64 MFMA (pwdf_stats.pairG_head):
                         the FP32 rounding then scales with the tail's weights */
} pwdf_precision;

/* What pwdf_build_j writes into J(k) (pwdf_set_jk_layout). */
typedef enum {
  PWDF_JK_FULL = 0,    /* every element of J(k): zeros off the pair support (default) */
  PWDF_JK_SUPPORT = 1, /* only the elements on the pair support (pwdf_stats.jk_support per k
                          and density); the others are never written, so the caller clears
                          J(k) once and keeps the buffer */
  PWDF_JK_PACKED = 2   /* the support elements only, packed: J(k) is complex128
                          [ndm][nk][jk_support] in the element order of
                          pwdf_get_jk_support */
} pwdf_jk_layout;

/* How the D(k) of pwdf_build_j / _graph / _noalloc, pwdf_get_rhoG and pwdf_grad
 * is laid out (pwdf_set_dk_layout). */
typedef enum {
  PWDF_DK_FULL = 0,  /* complex128 [ndm][nk][nbf][nbf], every element present (default) */
  PWDF_DK_PACKED = 1 /* complex128 [ndm][nk][jk_support]: only the elements of the J(k)
                        support, in the packed order of pwdf_get_jk_support (both
                        triangles; the packed J(k) of a build has this layout) */
} pwdf_dk_layout;

typedef struct {
  double eps_pair; /* pair screening on exp(-a_a a_b/p |A-B-L|^2); e.g. 1e-12 */
  double eps_G;    /* G cutoff |G| <= 2 omega sqrt(-ln eps_G); e.g. 1e-12 */
  double r_max;    /* centre-distance cap |A-B-L| <= r_max (Bohr); <= 0: off */
  int pair_gcut;   /* 1: every pair block (shell a, shell b, image) sees only the G
                      of the set inside its own cut radius, where the screening
                      objective 8 pi eta G (4 pi/G^2) e^{-G^2/4w^2} |F|_inf(G),
                      eta = [1/p + 1/w^2]^-1, of its most compact primitive pair
                      falls below eps_G (section "Integral screening", eqs. "AFT
                      screening obj", "eta_munu"; |F|_inf over the Cartesian
                      components with G along x, y, z); 0: every pair sees the
                      whole set */
  double alpha_cut; /* > 0: compact/diffuse classification (section "Density
                      classification: compact and diffuse"; eq. "cd cutoff" sets
                      alpha_cut = omega^2/2).  A primitive pair whose two exponents
                      both lie below alpha_cut is diffuse (DD); every interaction
                      with a DD side then takes the full-range kernel 4 pi/G^2:
                        V_C = v rho_C + (4 pi/G^2) rho_D   for compact pairs,
                        V_D = (4 pi/G^2)(rho_C + rho_D)    for DD pairs,
                        E_J = 1/2 Omega sum_G [rho_C V_C(-G) + rho_D V_D(-G)],
                      rho_C / rho_D the parts of rho from compact / DD pairs.  DD
                      pairs see the whole G set (no per-pair cut) and are
                      evaluated in FP64 in both precision forms; J, E_J, the
                      gradient and pwdf_get_rhoG (rho_C + rho_D) follow.  <= 0:
                      off.  Must be finite (PWDF_EINVAL) */
  int dd_gpw;       /* with alpha_cut > 0: 1 takes the DD pairs' density and J through
                      a real-space grid (GPW, appendix "Evaluation of density on
                      real space grid (GPW)"): rho_D(r) collocated on N1 x N2 x N3
                      points along the lattice vectors, N_i = 2 ceil(1.25 M_i) + 1
                      for the largest |n_i| = M_i of the G set, transformed onto
                      the G set by separable sums; V_D(G) back onto the grid and
                      integrated against each DD pair density into J(L).  Equal to
                      the analytic route up to the grid's aliasing (vectors beyond
                      the cutoff sphere).  The gradient keeps the analytic DD
                      moments.  0: analytic transforms of the DD pairs */
} pwdf_screen;

typedef struct {
  int64_t npairs_by_class[16]; /* unique primitive pairs per (la,lb), index la*4+lb (la >= lb) */
  int64_t nG;       /* |G set| (both G and -G); the kernels walk nG/2 of them */
  int64_t npairs;   /* unique primitive pairs (a,b,L) ~ (b,a,-L) counted once */
  int64_t nbf, nk, nimg, nblocks, nseg;
  double pairG_evals; /* per build and density: 2 passes x the G each unique pair sees
                         (npairs x nG/2 without per-pair cuts) */
  double t_us[8];     /* reserved */
  int64_t seg_len;    /* line-segment length of the current launch shapes (pwdf_query) */
  int64_t fork;       /* 1: independent launches of a pass overlap on internal streams;
                         0: they follow each other on the caller's stream (pwdf_query) */
  int64_t jk_support; /* matrix elements (mu,nu) of J(k) on the pair support (both
                         triangles): what a build writes per k and density in the
                         PWDF_JK_SUPPORT layout */
  int64_t dk_support; /* matrix elements of D(k) a build reads per k and density (one
                         of (mu,nu), (nu,mu) for each support pair of elements; in
                         the packed D(k) layout, pwdf_query: the packed ones) */
  int64_t jk_layout;  /* current pwdf_jk_layout (pwdf_query) */
  int64_t nG_head;    /* G vectors of the half space in the head (v(G) >= 2^-7 max v) */
  double pairG_head;  /* per build and density: the part of pairG_evals on the head G;
                         the FP32-MFMA form evaluates it with FP64 tiles */
  int64_t npairs_dd;  /* unique DD primitive pairs (pwdf_screen.alpha_cut); pairG_evals
                         counts them over the whole half space in both passes */
  int64_t gpw_grid[3]; /* GPW route (pwdf_screen.dd_gpw): grid points along a1, a2, a3
                          (0 when the DD pairs take the analytic route) */
} pwdf_stats;

/*
 * Build the plan for one geometry: reciprocal lattice, G set (walked as lines
 * in relative coordinates), screened unique primitive pairs sorted by class,
 * phase tables, and every device workspace for up to max_ndm densities per
 * call.  Passage: section "Long-range contributions" and section "Integral
 * screening" (pair list), appendix "Cartesian coordinates and relative
 * coordinates" (B, relative coordinates).
 *   lattice[9]     host, row-major rows a1,a2,a3; det must be nonzero.
 *   natm, xyz      host, natm x 3 Bohr; used as given (no wrapping).
 *   nshell         number of shells; shell_atom/shell_l/shell_nprim host [nshell];
 *                  0 <= shell_l <= 3; shell_nprim >= 1.
 *   exps, coefs    host, sum(shell_nprim) primitives in shell order; exps > 0.
 *   kmesh[3]       host, each >= 1, with (n1+n2+n3) lcm(n1,n2,n3) <= 1024
 *                  (PWDF_EUNSUPPORTED otherwise: the phase table lives in LDS).
 *   omega          range-separation parameter > 0 (Bohr^-1).
 *   screen         host; eps_pair, eps_G in (0, 1).
 *   prec           PWDF_FP64 or PWDF_FP32_MFMA.
 *   max_ndm        largest ndm accepted by later calls (>= 1).
 *   device         HIP device ordinal.
 * On success *out is a new context (free with pwdf_destroy).  PWDF_EINVAL also
 * when no G vector lies in the cutoff sphere (0 < |G| <= Gcut); the screened
 * pair list always holds at least the on-site pairs (K = 1).  PWDF_EUNSUPPORTED
 * when a pair is so diffuse (small a_a + a_b = p) that Gcut^2/4p or the step
 * ratio of the G-line recurrence exceeds 650: its Gaussian factors would
 * overflow or underflow in FP64 (message names p).
 */
pwdf_status pwdf_create(pwdf_ctx **out, const double lattice[9], int natm, const double *xyz,
                        int nshell, const int *shell_atom, const int *shell_l,
                        const int *shell_nprim, const double *exps, const double *coefs,
                        const int kmesh[3], double omega, const pwdf_screen *screen,
                        pwdf_precision prec, int max_ndm, int device);

/* Sizes and counts of the plan (host struct, filled).  PWDF_EINVAL for a NULL
 * ctx (message via pwdf_last_error(NULL)) or a NULL out. */
pwdf_status pwdf_query(const pwdf_ctx *ctx, pwdf_stats *out);

/*
 * Choose what later builds write into J(k) (pwdf_jk_layout).  Both layouts hold
 * the same values on the pair support (eq. "FT of J": J(k) is a sum over the
 * images of the screened pairs, so elements no pair block touches are exactly
 * zero).  PWDF_JK_SUPPORT skips those zeros: for a cell whose support is a small
 * share of nbf^2 (a slab with vacuum) the zero stores would otherwise dominate
 * the launch.  The caller must then clear J(k) once (the library never writes
 * the other elements, in any call).  A cached graph is dropped when the layout
 * changes.  Host only; PWDF_EINVAL for an unknown layout.
 */
pwdf_status pwdf_set_jk_layout(pwdf_ctx *ctx, int layout);

/*
 * FP32-MFMA form: the G vectors whose Coulomb weight v(G) = 4 pi e^{-G^2/4w^2}/G^2
 * is at least `weight` times the largest one (a ball around G = 0: the part of
 * the sum of eq. "Ewald J" that carries most of the energy) are contracted with
 * FP64 tiles on FP64 MFMA, the others with FP32 tiles.  A smaller weight moves
 * more of the pair-G work into FP64 (pwdf_stats.nG_head, pairG_head) and lowers
 * the FP32 rounding error of E_J and J; weight -> 0 takes every G in FP64.
 * Default 2^-20.  weight in (0, 1] (PWDF_EINVAL otherwise).  The context's device
 * workspaces are rebuilt for the new split (this call allocates and synchronises
 * the device; a cached graph is dropped; the launch shapes of the last
 * pwdf_autotune are kept, so tune again for the best ones).  The FP64 form only
 * reports the counts.
 */
pwdf_status pwdf_set_fp32_head(pwdf_ctx *ctx, double weight);

/*
 * D(k) layout of the calls that read a density (pwdf_dk_layout; default
 * PWDF_DK_FULL).  With PWDF_DK_PACKED a density is passed as the values of
 * D(k) on the J(k) support only, in the packed element order of
 * pwdf_get_jk_support: the D(k) -> D(L) phase sums (eq. "FT for D") then read
 * whole runs of each packed row (of the two Hermitian partners (mu, nu) and
 * (nu, mu) the one with shell(mu) <= shell(nu)) instead of a few elements per
 * row of the dense matrix.  Every D(L) value a build forms lies on that support,
 * so both layouts give the same J(k) and E_J up to rounding (the two read
 * opposite partners of some pairs: D(k) is taken as Hermitian).  A cached graph
 * is dropped when the layout changes.  Errors: PWDF_EINVAL (NULL ctx, unknown
 * layout).  Host only.
 */
pwdf_status pwdf_set_dk_layout(pwdf_ctx *ctx, int layout);

/*
 * Element order of the packed J(k) layout: for i < pwdf_stats.jk_support, the
 * i-th packed value of every (density, k) plane is J_{mu[i], nu[i]}(k).  mu and
 * nu are host arrays of jk_support ints (either may be NULL).  The elements are
 * the support of eq. "FT of J" (both triangles); the ones summed by one thread
 * come first in ascending row-major order, the ones with more than 8 lattice
 * image classes (summed by one wave each) follow.  Host only.
 */
pwdf_status pwdf_get_jk_support(const pwdf_ctx *ctx, int *mu, int *nu);

/*
 * Input check of the calls made since the previous check: the D(k) -> D(L)
 * launch of every build / gradient / rho call sets a device flag when a phase
 * sum over the D(k) values of a support element is not finite (a NaN or inf in
 * D(k)).  This call synchronises `stream`, reads and clears the flag, and
 * returns PWDF_ENONFINITE (with a message) when it was set, else PWDF_OK.  The
 * enqueueing calls cannot report it themselves: they return before the device
 * has read D(k).
 */
pwdf_status pwdf_check_input(pwdf_ctx *ctx, void *stream);

/* Host-only plan: validates the same arguments as pwdf_create, builds the G set
 * and the unique screened pair list on the host (no device is touched) and
 * fills *out.  Section "Integral screening" (pair list).  Errors as for
 * pwdf_create; the message is read with pwdf_last_error(NULL). */
pwdf_status pwdf_plan_stats(const double lattice[9], int natm, const double *xyz, int nshell,
                            const int *shell_atom, const int *shell_l, const int *shell_nprim,
                            const double *exps, const double *coefs, const int kmesh[3], double omega,
                            const pwdf_screen *screen, pwdf_stats *out);

/*
 * Long-range J for ndm densities: D(k) -> D(L) on the pair support (eq. "FT for
 * D"), per-pair density transform (algorithm "density matrix transformation"),
 * rho(G) (algorithm "non-ortho rho eval"), V(G) and E_J, J from V (algorithm
 * "non-ortho J eval"), back transform (algorithm "J matrix transformation")
 * and J(L) -> J(k) (eq. "FT of J").
 *   ndm   1 <= ndm <= max_ndm.
 *   Dk    device, complex128 [ndm][nk][nbf][nbf], Hermitian per k; read only;
 *         or [ndm][nk][jk_support] in the packed D(k) layout (pwdf_set_dk_layout).
 *   Jk    device, same layout; every element written (zeros off the pair support),
 *         or only the elements on the pair support (pwdf_set_jk_layout); packed
 *         layout: complex128 [ndm][nk][jk_support] (pwdf_get_jk_support).
 *   EJ    device, double [ndm]; written with E_J of each density.
 *   stream  hipStream_t or NULL.
 * Dk and Jk must not overlap.  Enqueue only.
 */
pwdf_status pwdf_build_j(pwdf_ctx *ctx, int ndm, const double *Dk, double *Jk, double *EJ,
                         void *stream);

/*
 * pwdf_build_j replayed as a HIP graph: the first call with a given
 * (ndm, Dk, Jk, EJ) captures the whole launch sequence (fork/join branches
 * included) on an internal stream, instantiates it and keeps it in the context;
 * this and later calls with the same arguments launch the instantiated graph on
 * `stream` (one launch instead of about a dozen kernel launches).  Results
 * equal those of pwdf_build_j bit for bit (same kernels, same shapes).  A call
 * with other arguments,
 * pwdf_autotune or pwdf_destroy drops the cached graph.  The graph holds kernel
 * launches and event dependencies only (no memset or copy nodes).
 * Errors: as pwdf_build_j; PWDF_ESTATE while profiling is enabled.
 */
pwdf_status pwdf_build_j_graph(pwdf_ctx *ctx, int ndm, const double *Dk, double *Jk, double *EJ,
                               void *stream);

/*
 * pwdf_build_j for callers that cannot allocate device memory at all (code
 * being captured into a HIP graph, tight serving loops, hosts that forbid
 * hipMalloc after start-up): the same launch sequence and results as
 * pwdf_build_j (bit for bit), but every per-call workspace of the build
 * (D(L) / J(L) blocks, transform coefficients, moment and partial-row arrays,
 * rho, V, energy partials, folded J, FP32-MFMA operands) lives in one static
 * device array of the library, 64 MiB per device, held by every device the
 * library is loaded on until the process ends.  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine); the context's own
 * allocations from pwdf_create (plan tables) are used as they are.
 *   Arguments, layouts and errors as pwdf_build_j, plus PWDF_EUNSUPPORTED
 *   (message states the bytes needed) when ndm densities of this plan need
 *   more workspace than the static array holds.
 * Every call on one device shares that device's array, whatever the context:
 * calls that overlap in time on one device (other streams, other threads, a
 * graph replay racing an eager call) race on it, so order them on one stream.
 * The array keeps the previous call's contents; the call clears what must
 * start at zero itself (with a kernel, so the call can be captured).
 */
pwdf_status pwdf_build_j_noalloc(pwdf_ctx *ctx, int ndm, const double *Dk, double *Jk, double *EJ,
                                 void *stream);

/*
 * rho(G) of the last computation path for diagnostics: runs the D(k) -> rho(G)
 * part of pwdf_build_j for ndm densities and writes, for the nG/2 vectors of
 * the half space the kernels walk (rho(-G) = conj rho(G)),
 *   rhoG    device, complex128 [ndm][nG/2]
 *   miller  host, int [nG/2][3] Miller indices n (G = B n) in the same order
 *           (may be NULL; filled from the plan before the call returns).
 * rhoG is written on the stream (asynchronous, like pwdf_build_j).
 */
pwdf_status pwdf_get_rhoG(pwdf_ctx *ctx, int ndm, const double *Dk, double *rhoG, int *miller,
                          void *stream);

/*
 * Real-space form of the energy, E_J^(R) = 1/2 sum over (a, b, L) of D_ab(L) J_ab(L)
 * (section "Long-range contributions": the energy as the contraction of the
 * real-space density and Coulomb blocks), from the D(L) and J(L) blocks that the
 * last pwdf_build_j or pwdf_build_j_graph call on ctx left in its workspace.  It
 * equals the E_J of that call (the G-space sum 1/2 Omega sum_G v |rho|^2, and its
 * compact/diffuse form) up to rounding, in either precision form: a cross-check
 * of the whole path rather than a second result.
 *   ndm  1 .. the ndm of that call: the first ndm densities.
 *   ER   device, double [ndm], written.
 * Same stream as the build (or ordered after it).  PWDF_ESTATE when the
 * workspace holds no such blocks: no build yet, fewer densities, or another call
 * since (pwdf_build_j_noalloc, pwdf_get_rhoG, pwdf_grad, pwdf_autotune,
 * pwdf_set_fp32_head replace them).
 */
pwdf_status pwdf_energy_real(pwdf_ctx *ctx, int ndm, double *ER, void *stream);

/*
 * Nuclear gradient dE_J/dR_A at fixed D(k), fixed pair list and fixed G set
 * (derivative of the pair transform with respect to the Gaussian centres,
 * eq. "cart gaussian function" and eq. "FT of cart Gaussians").
 *   Dk    device, as in pwdf_build_j.
 *   dEdR  device, double [ndm][natm][3], written.
 *   EJ    device, double [ndm] or NULL; written with E_J when not NULL.
 * The geometry is the one given to pwdf_create.
 */
pwdf_status pwdf_grad(pwdf_ctx *ctx, int ndm, const double *Dk, double *dEdR, double *EJ,
                      void *stream);

/* Pick launch shapes by timing candidates on the device for ndm densities:
 * the line-segment length (4, 5, 8 or 16 points; 4 or 8 for the FP32-MFMA
 * form) jointly with a common multiplier (1/2, 1 or 2) of the default number of
 * pair chunks of the rho pass and of segment chunks of the J pass, by the wall
 * time of the transform .. back-transform launches (FP64: captured as a graph
 * and replayed; FP32-MFMA form: eager launches, segment length first, then the
 * multiplier).  The FP32-MFMA form (one launch per angular class L) then lets
 * each class keep the multiplier (1/4 .. 4) of its shortest launch, and keeps
 * that result only if it also wins overall; the FP64 form tries the J pass's
 * multiplier at 1/2 and 2 and the rho pass's at 3/4 and 3/2 of the chosen one,
 * each kept only if at least 1 % faster, then the classes L >= 3 apart from
 * L <= 2 at 1/2 and 2.  Last, the independent launches of a pass either overlap
 * on the internal streams or follow each other on the caller's stream,
 * whichever replays faster (pwdf_stats.fork); the FP32-MFMA form first times
 * its per-class launches one at a time and also tries them overlapping in the
 * order of those times (longest first, each onto the least-loaded stream).
 * Timing runs on
 * an internal stream over zero D(L) and does not touch caller buffers.  The
 * device workspaces are rebuilt for the chosen shapes (this call allocates),
 * a cached graph is dropped and profiling counters are reset.  Results of later
 * calls agree with the untuned ones to rounding (summation order changes).
 * cache_path: text file of "key seg_len mrho[0..7] mj[0..7] fork lpt
 * cost[4][0..7]" lines (fork may be absent: 1; lpt and the launch times in ms
 * of the FP32-MFMA form's rho tail, rho head, J tail and J head launches may be
 * absent: class order) keyed by
 * arch, precision, nG, pair count, nbf, nk and ndm; an entry found there is
 * applied without timing (PWDF_EINVAL if its segment length is not one listed
 * above for the context's form), a new result is appended.  NULL: no
 * persistence.
 * Synchronous. */
pwdf_status pwdf_autotune(pwdf_ctx *ctx, int ndm, const char *cache_path);

/* Diagnostics: per-launch HIP-event timing on the caller's stream.
 * pwdf_profile_enable(ctx, 1) resets the counters and brackets every later
 * kernel launch of ctx with a pair of events on the stream it runs on
 * (creating events as needed, so keep it off under graph capture);
 * pwdf_profile_read synchronises on the recorded events and returns, per
 * kernel name, the launch count, the summed milliseconds and the summed work
 * units (algorithmic flops for the FP64 pair-G launches rho_lo/hi and
 * jpass_lo/hi, 8(L+1)+4 per unique pair, G of the half space and density;
 * pair-G evaluations for the FP32 launches rho_mfma_L* / jpass_mfma_L*; D(k) values read for
 * phase_d (elements on the pair support x Nk), J(k) values written for phase_j,
 * algorithmic flops for transform / back: two per term of the E-coefficient
 * contraction sum_ab D_ab E^x E^y E^z and per entry of the Hermite -> monomial
 * blocks, per pair and density).
 * out may be NULL to query the count; *n receives the number of names. */
typedef struct {
  char name[32];
  int64_t launches;
  double ms;
  double units;
} pwdf_kprof;
pwdf_status pwdf_profile_enable(pwdf_ctx *ctx, int on);
pwdf_status pwdf_profile_read(pwdf_ctx *ctx, pwdf_kprof *out, int max, int *n);

/* Message of the last failure on ctx (NULL: the last failure of this thread without a context). */
const char *pwdf_last_error(const pwdf_ctx *ctx);

/* Free the plan and all device workspaces; NULL is a no-op. */
void pwdf_destroy(pwdf_ctx *ctx);

/*
 * Test hooks of the library's device allocations (every plan upload and
 * workspace of every context goes through one allocator; the static scratch of
 * pwdf_build_j_noalloc is not an allocation).
 * pwdf_debug_fail_alloc(after): after >= 0 lets that many further allocations
 * succeed and fails every one after them with an out-of-memory error until the
 * next call; after < 0 turns the failures off (the default).  A setup that fails
 * returns PWDF_ENOMEM and releases what it had allocated: pwdf_create then
 * returns no context; a context whose re-setup failed (pwdf_autotune,
 * pwdf_set_fp32_head) answers PWDF_ESTATE to device work until pwdf_destroy.
 * pwdf_debug_live_allocs(): device allocations currently held by all contexts.
 * Process-wide; not for use while other threads create or tune contexts.
 */
void pwdf_debug_fail_alloc(int after);
int64_t pwdf_debug_live_allocs(void);

#ifdef __cplusplus
}
#endif
#endif /* PWDF_H */
