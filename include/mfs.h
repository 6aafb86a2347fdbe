/*
 * libmfs -- MI355X (gfx950) implementation of the hot path of the
 * axisymmetric method-of-fundamental-solutions (MFS) solver for acoustic
 * scattering from doubly-periodic arrays of axisymmetric obstacles
 * (Liu & Barnett, J. Comput. Phys. 2016).
 *
 * Conventions shared by every entry point
 *  - Every call returns mfs_status; no C++ exception crosses this ABI.  On a
 *    non-zero status mfs_last_error() returns a thread-local message.
 *  - Complex numbers are mfs_c128 = two doubles (re, im), the layout of
 *    torch.complex128 and of C99 double _Complex.
 *  - "host" pointers are read (or written) during the call; the caller keeps
 *    ownership.  "dev" pointers are caller-owned device memory on the
 *    context's GPU, 16-byte aligned and contiguous; work on them is queued on
 *    `stream` (a hipStream_t, NULL = the legacy default stream) and they must
 *    stay valid until that stream has been synchronised.
 *  - Library-owned objects (mfs_ctx, mfs_op) hold all factor storage and are
 *    released with the matching mfs_destroy_* call.
 *  - Mode arrays use FFT bin order: bin b (0 <= b < P) holds the azimuthal
 *    mode n = b for b <= P/2 and n = b - P above, n = -P/2+1..P/2 (Sec. 3,
 *    after eq. (fhat)).  A mode-n coefficient multiplies a field varying as
 *    e^{+i n phi}.  Angles are phi_l = 2 pi l / P, l = 0..P-1.
 *  - Calls on one context are not thread safe; use one context per thread
 *    or an external lock.
 */
#ifndef MFS_H
#define MFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MFS_OK = 0,
  MFS_EINVAL = 1,   /* bad argument; nothing was written                     */
  MFS_ENOMEM = 2,   /* device or host allocation failed                       */
  MFS_EDEVICE = 3,  /* a HIP call failed                                      */
  MFS_ENOTCONV = 4, /* GMRES hit maxit, or a Jacobi SVD its sweep cap;
                       results hold the last iterate                         */
  MFS_ESTATE = 5,   /* call out of order (e.g. apply before factor)          */
  MFS_EBUSY = 6
} mfs_status;

typedef struct { double re, im; } mfs_c128;

typedef struct mfs_ctx mfs_ctx;
typedef struct mfs_op mfs_op;

/* One axisymmetric body and its one-body discretisation (Sec. 3).
 * M collocation points (rho_m, z_m) on the generating curve with outward unit
 * normals (nrho_m, nz_m); N MFS sources (srho_j > 0, sz_j) inside the body;
 * P azimuthal modes (even, >= 2); q trapezoid nodes for the ring-kernel fill
 * (eq. (ptr); even, q >= P); k > 0 the wavenumber.  M >= N.
 * km = 0: sound-hard body (eq. (neu)).  km > 0: transmission (eqs.
 * (helmi)-(neup1.4), Sec. 3.4) with interior wavenumber km; the interior
 * field is a second ring-source sum at km with the N sources
 * (srho_out, sz_out) outside the body (tau negated).  The per-mode system is
 * then 2M x 2N (eq. (trans)): rows [values; normal derivatives] of the M
 * collocation points, columns [exterior; interior] coefficients, and every
 * "[..][P][M]" surface array and "[..][P][N]" coefficient array below has
 * 2M and 2N entries per mode instead. */
typedef struct {
  int32_t M, N, P, q;
  double k;
  const double *rho, *z, *nrho, *nz; /* host [M] */
  const double *srho, *sz;           /* host [N] */
  double km;                         /* 0, or the interior wavenumber       */
  const double *srho_out, *sz_out;   /* host [N], km > 0 only               */
} mfs_body;

/* Polar generating curve r(t) = a (1 + eps cos(j t)), rho = r sin t,
 * z = r cos t, t in [0, pi] (Sec. 3); sources at t_j = pi (j - 1/2)/N moved
 * into the body by complexification Z(t_j - i tau), Z = rho + i z (Sec. 3.2,
 * method (c)); collocation colloc = 0: t_m = pi (m - 1/2)/M,
 * colloc = 1: Gauss-Legendre nodes in t. */
typedef struct {
  double a, eps;
  int32_t j;
  int32_t colloc;
  int32_t M, N;
  double tau;
} mfs_polar_spec;

/* Cup generating curve of Fig. 1(c): with u = pi - t, x = u - pi/2,
 *   r = 1 - half erf(x/half),
 *   theta = b - half + 2 (1 - (b - half)/pi) s(x),
 *   s(x) = x erf(x/half) + (half/sqrt(pi)) e^{-x^2/half^2}  (rounded |x|),
 *   rho = c r sin theta, z = c r cos theta,  c = outer/(1 + half):
 * a shell of half-thickness `half` about the unit sphere with an opening of
 * half-angle b about +z, scaled to outer radius `outer`; t = 0 is the inner
 * bottom pole.  Sources, collocation and tau as for mfs_polar_spec (the
 * complex erf of the sources is evaluated for |tau| <= half; tau < 0 puts the
 * sources outside, for the interior field of a transmission body). */
typedef struct {
  double outer, half, b;
  int32_t colloc;
  int32_t M, N;
  double tau;
} mfs_cup_spec;

/* Rectangular lattice e_x, e_y; unit cell |z| <= z0; periodizer: harmonic
 * degree p, Rayleigh-Bloch cutoff kappa_x^2 + kappa_y^2 <= (pi N0)^2, M1 x M1
 * Gauss nodes per wall (M1 even) (Sec. 4, Sec. 4.1). */
typedef struct {
  double ex, ey, z0;
  int32_t p;
  double N0;
  int32_t M1;
} mfs_lattice;

/* Incident plane wave from above, k_vec = k (sin th cos ph, sin th sin ph,
 * -cos th) (eq. (ui)). */
typedef struct { double theta, phi; } mfs_wave;

/* Per-wave result of mfs_solve_incident.  The caller provides the arrays
 * and their capacities; the library fills them.  Bragg orders are listed by
 * m, then n (m, n, kappa_z as in eqs. (rb1)-(rb2)). */
typedef struct {
  int32_t iters;          /* GMRES iterations                                 */
  double resid;           /* final relative residual of eq. (iter)            */
  int32_t norders;        /* number of Bragg orders kept                      */
  int32_t cap_orders;     /* capacity of m, n, kz, a, b                       */
  int32_t *m, *n;         /* host [cap_orders]                                */
  mfs_c128 *kz;           /* host [cap_orders] kappa_z (+real or +imag)      */
  mfs_c128 *a, *b;        /* host [cap_orders] upward / downward amplitudes   */
  mfs_c128 *field;        /* host [ntargets] scattered field u at targets     */
  double eps_flux;        /* energy-flux defect (Sec. 5)                     */
  int32_t q_rank;         /* numerical rank kept in Q^+                       */
  int32_t nq_cols;        /* columns of Q                                     */
} mfs_result;

/* Timing of the last mfs_solve_incident stages, milliseconds (HIP events on
 * the operator's stream). */
typedef struct {
  double rhs, periodizer, gmres, recover, total;
  double nsum_avg;        /* mean duration of one neighbour-sum launch (the
                             surface sums of A_else and the wall sums of C)   */
  int32_t nsum_launches;
  double jacobi_ms;       /* Jacobi sweeps of the periodizer's pseudoinverse   */
  int32_t jacobi_launches;
  double jacobi_bytes;    /* algorithmic HBM bytes of those launches: every
                             block-pair task reads its columns of G, a task
                             that rotated also writes them and reads and
                             writes its columns of V                          */
  double jacobi_flops;    /* algorithmic FP64 flops: the Hermitian Gram matrix
                             of every task, and the rotation product applied
                             to G and V by the tasks that rotated             */
  double near_fill_ms;    /* filling the dense near field (0 if on the fly)  */
  double near_bytes;      /* mean dense near-field bytes streamed by one of
                             those launches (0 if evaluated on the fly)       */
  double near_alg_bytes;  /* the same without the padding of the last 64-target
                             tile of each group: the values the method needs */
  int32_t near_mode;      /* 0: sums evaluated on the fly (budget 0); 1: stored
                             near field; 2: on the fly because the stored field
                             did not fit the budget or the free device memory;
                             3: it did not fit, and the surface sums use
                             low-rank factors of the image blocks (the wall
                             sums on the fly); near_fill_ms is then the time
                             to build the factors (0 if an earlier solve on
                             the same lattice built them)                    */
  double q_qr_ms;         /* blocked Householder QR of the waves' Q (one batch) */
  double q_qr_flops;      /* its algorithmic flops, sum of 8 m n^2 - 8 n^3 / 3  */
  double q_post_ms;       /* the rest of Q^+: triangle inverse (or the SVD path)
                             and the explicit factors                         */
} mfs_solve_timing;

const char *mfs_last_error(void);
const char *mfs_version(void);

/* Create a context on HIP device `device`.  Allocates nothing large. */
mfs_status mfs_create(int device, mfs_ctx **out);
void mfs_destroy(mfs_ctx *ctx);

/* Device memory of the library.  Every device buffer of 1 MiB or more that
 * the library allocates comes from a per-device cache: a released buffer is
 * kept (after the device has finished the work queued before its release)
 * and handed to the next request of about its size, so repeated solves do
 * not return tens of GB to the driver and ask for them again.  At most half
 * of the device's memory is kept idle; a failed allocation first frees the
 * idle blocks and retries.
 *   mfs_memory_stats: bytes held by live library buffers (in_use), their
 *     largest value since the last mfs_memory_reset_peak (peak), and idle
 *     cached bytes (cached); any pointer may be NULL.
 *   mfs_release_cached_memory: return the idle cached blocks to the driver
 *     (for a caller that needs the memory for something else).
 * EINVAL for a device that does not exist. */
mfs_status mfs_memory_stats(int device, uint64_t *in_use, uint64_t *peak, uint64_t *cached);
mfs_status mfs_memory_reset_peak(int device);
mfs_status mfs_release_cached_memory(int device);

/* Host helper: geometry of a polar body, written into caller arrays
 * rho, z, nrho, nz [spec->M] and srho, sz [spec->N] (Sec. 3, Sec. 3.2). */
mfs_status mfs_polar_geometry(const mfs_polar_spec *spec, double *rho, double *z,
                              double *nrho, double *nz, double *srho, double *sz);

/* Host helper: geometry of the cup (Fig. 1(c)) into the same caller arrays.
 * EINVAL for outer <= 0, half outside (0, 1), b outside (0, pi), tau outside
 * [-half, half], M or N < 1, or colloc not 0/1; nothing is written then. */
mfs_status mfs_cup_geometry(const mfs_cup_spec *spec, double *rho, double *z,
                            double *nrho, double *nz, double *srho, double *sz);

/* (a) Modal fill (eqs. (ringkernelderiv), (ptr)): for each body, the P/2+1
 * distinct blocks A'_n, n = 0..P/2 (A'_{-n} = A'_n) of size M x N,
 *   A'_n[m, j] = (1/q) sum_{l=0}^{q-1} dG/dn_x((rho_m,0,z_m); y_j(2 pi l/q)) e^{-i n 2 pi l/q},
 * G = e^{ikR}/(4 pi R) (eq. (G)); for a transmission body the 2M x 2N blocks
 * [[A_n, -A^-_n], [A'_n, -A'^-_n]] of eq. (trans), A_n the value kernel
 * (eq. (ringkernel)) and the minus blocks at km from the exterior sources.
 * All bodies are filled in one persistent launch.  Host arrays are copied;
 * the operator owns the blocks.  Returns EINVAL for P odd, q < P, q odd,
 * M < N, srho <= 0, km < 0, missing exterior sources or non-finite input. */
mfs_status mfs_build_operator(mfs_ctx *ctx, const mfs_body *bodies, int32_t nbodies,
                              void *stream, mfs_op **out);
void mfs_destroy_op(mfs_op *op);

/* Copy the filled blocks of one body, before factorisation, to dev
 * out [P/2+1][N][M] (column-major M x N per mode n = 0..P/2; [2N][2M] for a
 * transmission body).  ESTATE after mfs_factor_modes (the blocks are
 * released). */
mfs_status mfs_op_blocks(const mfs_op *op, int32_t body, mfs_c128 *out, void *stream);

/* (b) Per-mode factorisation (Sec. 3 and Sec. 4.2): blocked Householder QR
 * A'_n = Q_n R_n, SVD of R_n by one-sided Jacobi, singular values below
 * rel_cutoff * s_max dropped; keeps U_n = Q_n W_n (M x r) and V_n S_n^+
 * (N x r) so that A'_n^+ x = V_n S_n^+ (U_n^* x) is applied without forming
 * the pseudoinverse.  Blocking until done.  ranks (host, optional) receives
 * the kept rank of each distinct block, [sum over bodies of P/2+1].
 * The blocked Jacobi (here and for the periodizer's Q^+ in
 * mfs_solve_incident) uses 32-column blocks once a batch's widest factor
 * has 2048 columns, 16-column blocks below; the environment variable
 * MFS_JACOBI_WIDE_MIN_COLS, read at every factorisation, moves that width
 * (a test of the wide path on small matrices sets it to 0).  The Jacobi
 * stops after 40 sweeps (MFS_JACOBI_MAX_SWEEPS, read at every
 * factorisation, lowers the cap); if some block still rotates then, the
 * factors of the last sweep are kept and ENOTCONV is returned.  ESTATE if
 * the operator is already factored. */
mfs_status mfs_factor_modes(mfs_op *op, double rel_cutoff, int32_t *ranks);

/* Stage times of the operator, milliseconds, measured with HIP events on the
 * operator's stream: ms[0] fill (mfs_build_operator), ms[1] QR and ms[2]
 * Jacobi truncation + explicit U (mfs_factor_modes; zero before it runs). */
mfs_status mfs_op_timing(const mfs_op *op, double *ms);

/* Singular values (descending) of the distinct blocks of one body, host
 * out [P/2+1][N] ([P/2+1][2N] for a transmission body).  ESTATE before
 * mfs_factor_modes.  All zero when the environment set MFS_OPINV=cod for
 * the factorisation: the truncated pseudoinverses were then taken as
 * complete orthogonal decompositions (pivoted QR of the triangle, cut where
 * the trailing block's Frobenius norm falls to rel_cutoff times the largest
 * singular value, then the inverse of its LQ factor), which form none; the
 * ranks are those kept by that cut.  The periodizer's Q takes that form by
 * default from 4096 kept columns on (MFS_QPINV=svd or cod decides). */
mfs_status mfs_op_singular_values(const mfs_op *op, int32_t body, double *out);

/* Layouts of mfs_apply_solution_op. */
enum {
  MFS_LAYOUT_MODES = 0,  /* in: [nrhs][P][M] mode coefficients (FFT bin order);
                            out: [nrhs][P][N] mode coefficients c_n           */
  MFS_LAYOUT_ANGLE = 1,  /* in only: [nrhs][M][P] samples f(rho_m, phi_l, z_m)
                            at the P angles phi_l = 2 pi l / P (l contiguous) */
  MFS_LAYOUT_POINTS = 2  /* out only: [nrhs][P][N] point strengths
                            sigma_jl = (1/P) sum_n c_nj e^{+i n phi_l} of the
                            sources at the P angles (the sigma input of
                            mfs_neighbour_sum with qs = P)                  */
};

/* (c) Solution-operator apply (Sec. 3 eq. (linsys) and Sec. 4.2): for every
 * mode, c_n = A'_n^+ f_n with the truncated factors of mfs_factor_modes.
 * With in_layout ANGLE the library first takes the angle DFT
 * f_n = (1/P) sum_l f(phi_l) e^{-i n phi_l} (eq. (fhatquad), q = P); with
 * out_layout POINTS it returns the point strengths of the P-angle source
 * rings (the point-source form of Sec. 4.1) instead of the modes.  For a
 * transmission body M and N read 2M and 2N in the MODES and ANGLE layouts
 * (rows [values; normal derivatives], columns [exterior; interior]), while
 * POINTS holds the exterior sources' strengths, [nrhs][P][N].
 * in, out: dev, caller-owned, on the context's device.  An ANGLE input or a
 * POINTS output needs an intermediate [nrhs][P][M] or [nrhs][P][N] buffer,
 * taken from the library's device cache; the per-mode work buffer belongs to
 * the operator.  Asynchronous on `stream`.  ESTATE before mfs_factor_modes;
 * EINVAL for an unknown layout (nothing written). */
mfs_status mfs_apply_solution_op(const mfs_op *op, int32_t body, int32_t nrhs,
                                 const mfs_c128 *in, int32_t in_layout,
                                 mfs_c128 *out, int32_t out_layout, void *stream);

/* mfs_apply_solution_op without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, layouts, results and
 * errors as mfs_apply_solution_op; the caller still provides in and out.
 * Its work memory (the per-mode work buffer, nd x 32 x N complex values for
 * nd = P/2+1 distinct modes, plus the [nrhs][P][M] / [nrhs][P][N]
 * intermediates of an ANGLE input / POINTS output) lives in a static 64 MiB
 * device array that every GPU the library runs on holds until the process
 * ends; a call that would need more returns EINVAL and writes nothing.  All
 * calls on one GPU share that array, which keeps the last call's contents:
 * calls that overlap on one GPU (on different streams, or from different
 * threads) race, so serialise them (one stream, or an external lock). */
mfs_status mfs_apply_solution_op_noalloc(const mfs_op *op, int32_t body, int32_t nrhs,
                                         const mfs_c128 *in, int32_t in_layout,
                                         mfs_c128 *out, int32_t out_layout, void *stream);

/* Right-hand side of eq. (linsys): f = -du^i/dn at the P x M surface points
 * then f_hat_n = (1/P) sum_l f(phi_l) e^{-i n phi_l} (eq. (fhatquad), q = P).
 * For a transmission body [f_hat; f_hat'] of eq. (trans): f = -u^i in rows
 * [0, M) and f' = -du^i/dn in rows [M, 2M) of every mode.
 * kvec: host [nwaves][3] wave vectors; out: dev [nwaves][P][M] ([..][P][2M]). */
mfs_status mfs_rhs_modes(const mfs_op *op, int32_t body, int32_t nwaves, const double *kvec,
                         mfs_c128 *out, void *stream);

/* Point-source form (Sec. 4.1): sigma_{jl} = (1/qs) sum_n c_{nj} e^{+i n 2 pi l/qs}
 * for qs >= P.  c: dev [nrhs][P][N] (for a transmission body [nrhs][P][2N],
 * of which the exterior coefficients, columns [0, N), are used);
 * sigma: dev [nrhs][qs][N]. */
mfs_status mfs_point_strengths(const mfs_op *op, int32_t body, int32_t nrhs, int32_t qs,
                               const mfs_c128 *c, mfs_c128 *sigma, void *stream);

/* Target sets of mfs_neighbour_sum. */
enum {
  MFS_TARGETS_SURFACE = 0, /* the P x M surface nodes, normal derivative, the
                              8 non-central images (A_else before its FFT)  */
  MFS_TARGETS_WALLS = 1,   /* the 8 M1^2 wall rows of C (eq. (full)), with the
                              3x3 cancellation of Sec. 4.1                  */
  MFS_TARGETS_USER = 2     /* user points, all 9 near copies                */
};

/* (c) Direct phased 3x3-neighbour Helmholtz sum (eqs. (A), (Phinear)) of the
 * qs x N point sources y_{jl} + a e_x + b e_y with strengths sigma and
 * weights alpha^a beta^b.
 *   sigma: dev [nrhs][qs][N] (qs = P for SURFACE and WALLS);
 *   ab:    host [nrhs][2] Bloch phases (alpha, beta);
 *   user:  host [nuser][6] (x, y, z, dx, dy, dz) for USER targets: the output
 *          is the value (want = 0) or the derivative along (dx,dy,dz)
 *          (want = 1);
 *   out:   dev [nrhs][ntargets] with ntargets = P*M (SURFACE, [l][m] order),
 *          8*M1*M1 (WALLS, row order of eq. (full)) or nuser (USER). */
mfs_status mfs_neighbour_sum(const mfs_op *op, int32_t body, const mfs_lattice *lat,
                             int32_t nrhs, int32_t qs, const mfs_c128 *sigma, const mfs_c128 *ab,
                             int32_t target_set, const double *user, int32_t nuser, int32_t want,
                             mfs_c128 *out, void *stream);

/* Free-space field u(x) = sum_{j,l} G(x, y_{jl}) sigma_{jl} of the qs-node
 * point form of mode coefficients c (dev [nrhs][P][N]; for a transmission
 * body the exterior columns of [nrhs][P][2N]) at host targets [ntargets][3]
 * outside the body; out: dev [nrhs][ntargets]. */
mfs_status mfs_field_free(const mfs_op *op, int32_t body, int32_t nrhs, int32_t qs,
                          const mfs_c128 *c, const double *targets, int32_t ntargets,
                          mfs_c128 *out, void *stream);

/* Interior field u^- of a transmission body (Sec. 3.4): the ring sources at
 * km from the exterior sources, coefficients the columns [N, 2N) of c
 * (dev [nrhs][P][2N]), qs-node point form, at host targets [ntargets][3]
 * inside the body; out: dev [nrhs][ntargets].  EINVAL for a sound-hard
 * body. */
mfs_status mfs_field_interior(const mfs_op *op, int32_t body, int32_t nrhs, int32_t qs,
                              const mfs_c128 *c, const double *targets, int32_t ntargets,
                              mfs_c128 *out, void *stream);

/* Near-field policy of later mfs_solve_incident calls on op.  The kernel
 * values of the neighbour sums (the 8 images of A_else on the surface nodes
 * and the images of the wall rows of C) depend on the body, the lattice and
 * k only, so a solve may fill them once in device memory and stream them in
 * every GMRES iteration instead of evaluating them (the paper keeps B and C
 * dense in RAM and applies A_else by the FMM; on one GPU all three fit).
 * max_bytes bounds that storage: 0 evaluates the sums on the fly every
 * iteration; the default (UINT64_MAX) stores them whenever they fit with
 * 2 GiB of device memory to spare.  Results agree to rounding either way.
 * Both forms split the sources of every 64-target tile into slices (one
 * workgroup each, at least 256 sources a slice) aiming at 6144 workgroups
 * per sum; the environment variable MFS_NSUM_WORKGROUPS, read once per
 * process, sets another aim (slice count changes only the order in which
 * partial sums are added). */
mfs_status mfs_set_near_field_budget(mfs_op *op, uint64_t max_bytes);

/* (c) Periodic solve for nwaves incident waves (Sec. 4.2): per wave, fill and
 * factor Q = [S, -W], then GMRES on
 * eq. (iter) (I + A_else A_0^+ - B Q^+ C A_0^+) eta~ = f_hat, unrestarted from
 * zero, CGS2 orthogonalisation, stopping at ||r|| <= tol ||f_hat||;
 * eta = A_0^+ eta~, xi = -Q^+ C eta; the Bragg amplitudes a, b; the field
 * u at the host targets [ntargets][3] from eq. (urep) with q_field-node
 * point sources; eps_flux.  Blocking.
 * Q^+: the truncated SVD pseudoinverse (singular values below rel_cutoff
 * times the largest dropped) of Q with its columns scaled to unit norm, the
 * scaling folded back into the factors (Q^+ = D (Q D)^+).  When
 * ||R||_F ||R^{-1}||_F < 1/rel_cutoff for the triangle R of the QR of Q D,
 * no singular value can fall below the cutoff and Q^+ = D R^{-1} Q_1^*
 * is formed without the SVD.
 * Returns ENOTCONV if some wave hit maxit or its Q's Jacobi SVD its sweep
 * cap (the results hold the last iterate), EINVAL if a result's cap_orders
 * is too small (norders is set so the caller can retry).
 * timing (optional) receives stage times.  With the environment variable
 * MFS_PROGRESS set, the stages and every fifth GMRES iteration are reported
 * on stderr. */
mfs_status mfs_solve_incident(mfs_ctx *ctx, const mfs_op *op, int32_t body,
                              const mfs_lattice *lat, int32_t nwaves, const mfs_wave *waves,
                              double tol, int32_t maxit, double rel_cutoff,
                              const double *targets, int32_t ntargets, int32_t q_field,
                              mfs_result *res, mfs_solve_timing *timing);

/* ------------------------------------------------------------- serving
 * A server keeps the factored operator of one body and the lattice resident
 * and solves incident waves as they arrive (continuous batching): a fixed
 * pool of `slots` waves iterates in lockstep GMRES on eq. (iter), one batched
 * operator application per iteration for every wave in flight; a wave that
 * arrives is factored (its Q fill and truncated Q^+, Sec. 4.2) on a second
 * stream while the others iterate, joins the pool at the next iteration
 * boundary once a slot and memory are free, and leaves it when it converges
 * (its amplitudes and fields are then recovered as in mfs_solve_incident).
 * Every wave's arithmetic is independent of the others in the pool, so a
 * result is the same alone and in any mix (up to the rounding of its own Q
 * factorisation, which is batched with the waves admitted with it).  Two
 * host threads of the library drive the two streams. */
typedef struct mfs_server mfs_server;

typedef struct {
  int32_t slots;          /* waves iterating at once, 1..16                   */
  int32_t admit_batch;    /* waves factored together, 1..slots                */
  int32_t queue_cap;      /* pending requests before submit returns EBUSY     */
  double tol;             /* GMRES relative residual (eq. (iter))             */
  int32_t maxit;          /* GMRES iteration cap per wave                     */
  double rel_cutoff;      /* truncation of Q^+ (1e-10)                        */
  const double *targets;  /* host [ntargets][3] field points of every result  */
  int32_t ntargets;
  int32_t q_field;        /* point-source nodes of the field evaluation       */
  uint64_t hbm_budget;    /* device bytes the server may hold: the stored near
                             field, the slots' Krylov bases and Q factors and
                             the factorisation work of one admission group;
                             requests wait while it would be exceeded          */
} mfs_server_config;

/* Start a server on op (factored) and body for lattice lat.  Copies the
 * configuration and targets; fills the stored near field (within
 * hbm_budget) before returning.  EINVAL for bad sizes, ESTATE if op is not
 * factored, ENOMEM if the pool and one admission group do not fit. */
mfs_status mfs_server_create(mfs_ctx *ctx, const mfs_op *op, int32_t body, const mfs_lattice *lat,
                             const mfs_server_config *cfg, mfs_server **out);
/* Queue one incident wave; ticket receives its id.  Non-blocking; EBUSY if
 * queue_cap requests are already waiting. */
mfs_status mfs_server_submit(mfs_server *srv, const mfs_wave *wave, uint64_t *ticket);
/* Result of a finished request, as mfs_solve_incident would return it (res
 * arrays provided by the caller; EINVAL with norders set if cap_orders is
 * too small).  latency_ms (optional) receives completion minus submission
 * time.  EBUSY: not finished yet; EINVAL: unknown ticket (or already
 * collected); ENOTCONV: finished at maxit (res holds the last iterate);
 * EDEVICE: the server failed (mfs_last_error has the reason). */
mfs_status mfs_server_poll(mfs_server *srv, uint64_t ticket, mfs_result *res, double *latency_ms);
/* Requests waiting, being factored, iterating, and finished but not yet
 * collected (any pointer may be NULL). */
mfs_status mfs_server_stats(mfs_server *srv, int32_t *pending, int32_t *admitting, int32_t *iterating,
                            int32_t *finished);
/* Stop the server (requests not finished are dropped) and free it. */
void mfs_server_destroy(mfs_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* MFS_H */
