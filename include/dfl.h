/*
 * dfl.h -- C ABI of the MI355X (gfx950) deflated SAP-GCR Wilson-clover solver.
 *
 * The library solves the Dirac equation  D psi = eta  (arXiv:1605.00564,
 * section 2.2) for the O(a)-improved Wilson (clover) operator by GCR, right
 * preconditioned with the Schwarz alternating procedure (SAP), optionally
 * with block-local deflation, and drives the many truncated ("sloppy") and
 * few exact solves that all-mode averaging needs (section 2.1).
 *
 * Operator (the paper names it but does not write it out; the library uses
 * the kappa-normalised form):  M = A - kappa H  with
 *   (H psi)(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                     + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu),
 *   A(x) = 1 + i kappa c_sw sum_{mu<nu} sigma_{mu nu} Fhat_{mu nu}(x),
 *   Fhat_{mu nu} = (Q_{mu nu} - Q_{mu nu}^+)/8 (four plaquette leaves),
 * Euclidean chiral basis gamma_0 = [[0,-1],[-1,0]], gamma_k =
 * [[0,-i sigma_k],[i sigma_k,0]], sigma_{mu nu} = (i/2)[gamma_mu,gamma_nu].
 * The mass-normalised D = M / (2 kappa); solutions returned are M^{-1} b.
 *
 * Conventions shared by every entry point
 *   - dims = {T, X, Y, Z}; mu = 0 is time; site i = z + Z*(y + Y*(x + X*t)).
 *   - Vector buffers are caller-owned DEVICE pointers in the canonical layout
 *     [nrhs][V][4 spin][3 colour] of interleaved complex numbers, complex128
 *     for QCD_F64 and complex64 for QCD_F32 ("io" precision).  They must not
 *     alias each other unless a function says so.
 *   - Links are passed once, from HOST memory, as complex128 [V][4][3][3]
 *     (U_mu(x) links x to x+mu; SU(3) required because the reduced-precision
 *     copies store two rows and rebuild the third).
 *   - Every call is enqueued on the caller's HIP stream; calls that fill host
 *     arrays (info) synchronise that stream before returning.
 *   - Handles are library-owned; one host thread at a time per handle.
 *   - Return codes: 0 ok; QCD_NOCONV (1) = a solve did not reach its target
 *     (solution, iterations and residual are still written); negative values
 *     are errors, detailed by qcd_last_error().
 */
#ifndef DFL_H
#define DFL_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QCD_OK 0
#define QCD_NOCONV 1
#define QCD_EINVAL (-1)     /* null pointer, bad size or unsupported option */
#define QCD_EGEOM (-2)      /* block does not divide the lattice, odd block
                               extent, or an odd number of blocks in a direction */
#define QCD_ENOMEM (-3)     /* device allocation failed */
#define QCD_EHIP (-4)       /* HIP runtime error */
#define QCD_ESINGULAR (-5)  /* singular clover block, little-operator block or
                               rank-deficient deflation fields */
#define QCD_ENAN (-6)       /* NaN or Inf in an input or a norm */
#define QCD_ENOTSET (-7)    /* e.g. deflation requested but not set up */

typedef enum { QCD_F64 = 0, QCD_F32 = 1, QCD_F16 = 2, QCD_BF16 = 3 } qcd_prec;

/* Lattice, operator parameters and the Schwarz block grid.  The block grid
 * fixes the library's internal site order (block-major, parity split), so a
 * field handle serves one Schwarz block size; deflation uses it too unless
 * deflation_setup is given a larger multiple of it.  Each block
 * extent must be even and divide the lattice extent, and the number of
 * blocks in every direction must be even so that the two-colour checkerboard
 * of blocks (Omega, Omega*, section 2.2) closes periodically. */
typedef struct {
    int dims[4];     /* T, X, Y, Z */
    int block[4];    /* Schwarz block extents (and the default deflation block) */
    double kappa;
    double csw;
    int bc_t;        /* -1: antiperiodic in time (fermions), +1: periodic */
} qcd_lattice;

typedef struct qcd_field_s *qcd_field;
typedef struct qcd_dfl_s *qcd_dfl;

/* Error text for a return code, and the message of the last failure on the
 * calling thread (never NULL). */
const char *qcd_strerror(int code);
const char *qcd_last_error(void);

/* Build a field handle: copies links_host to the device, packs the storage
 * copies (FP64 full matrices; FP32, FP16 and BF16 with two rows), builds the
 * clover term A(x) from the clover leaves in FP64 and the inverse of A on
 * odd sites (needed by the even-odd block solves), then rounds both to the
 * reduced storage types.  Singular clover blocks give QCD_ESINGULAR. */
int qcd_field_create(const qcd_lattice *lat, const double *links_host, hipStream_t stream,
                     qcd_field *out);
/* Same, with the complex128 [V][4][3][3] links already in DEVICE memory
 * (caller-owned, only read during the call): everything after the links
 * reach HBM (site tables, packing, clover term, inverse) runs on the GPU. */
int qcd_field_create_device(const qcd_lattice *lat, const double *links_dev, hipStream_t stream,
                            qcd_field *out);
int qcd_field_destroy(qcd_field f);

/* out = M in for nrhs vectors (the Dirac operator of section 2.2).
 * io: QCD_F64 or QCD_F32 canonical vectors.  compute/storage:
 *   QCD_F64: FP64 links, clover and arithmetic;
 *   QCD_F32: FP32 links (two rows), clover and arithmetic;
 *   QCD_F16 / QCD_BF16: FP16 / BF16 links (two rows), FP16 clover, FP32
 *   arithmetic and FP32 vectors.
 * in and out must not overlap. */
int dirac_apply(qcd_field f, const void *in, void *out, int nrhs, qcd_prec io, qcd_prec storage,
                hipStream_t stream);

/* Same operator with explicit internal spinor storage on each side.
 * spinor_in / spinor_out: QCD_F64 (with FP64 storage only), QCD_F32, or
 * QCD_F16 = FP16 spinors with a per-site power-of-two scale (the site's
 * largest |re| or |im| is scaled into [2^14, 2^15) before rounding; 52
 * bytes per site), which needs QCD_F16 or QCD_BF16 operator storage.  The
 * input is rounded to spinor_in on the way in and the result to spinor_out
 * before it is returned; arithmetic is FP32 (FP64 with FP64 storage).
 * dirac_apply(...) equals dirac_apply_ex(..., v, v) with v = F64 for FP64
 * storage, else F32. */
int dirac_apply_ex(qcd_field f, const void *in, void *out, int nrhs, qcd_prec io, qcd_prec storage,
                   qcd_prec spinor_in, qcd_prec spinor_out, hipStream_t stream);

/* dirac_apply for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid allocation): the
 * same operator and arguments, with the input and output staged in the
 * library's internal layout in a static device array of 64 MiB per GPU
 * (held from the library's first use of that GPU until the process ends)
 * instead of workspace that grows on demand; no device memory is allocated
 * and no profiling events are created.  Staging needs 2 x nrhs x V x 96
 * bytes (FP32 vectors; 192 with FP64 storage); a call that needs more than
 * 64 MiB returns QCD_EINVAL.  Calls overlapping in time on one GPU share the
 * array and must not be issued (they race).  The field's device must be
 * current. */
int dirac_apply_noalloc(qcd_field f, const void *in, void *out, int nrhs, qcd_prec io, qcd_prec storage,
                        hipStream_t stream);

/* Schwarz preconditioner psi = M_SAP eta (section 2.2): ncy cycles starting
 * from psi = 0; each cycle visits all blocks of colour 0 (Omega) in
 * parallel, then all blocks of colour 1 (Omega*).  A block visit computes the
 * block residual eta - M psi with the current neighbour values, solves the
 * block equation with Dirichlet boundaries approximately by nmr
 * minimal-residual steps on the even-odd reduced block operator
 * A_ee - kappa^2 H_eo A_oo^{-1} H_oe, and adds the correction to psi. */
typedef struct {
    int ncy;           /* Schwarz cycles (the paper keeps 5) */
    int nmr;           /* minimal-residual steps per block solve */
    qcd_prec storage;  /* QCD_F64 (all FP64), QCD_F32, QCD_F16, QCD_BF16 (FP32 arithmetic) */
    qcd_prec vecs;     /* storage of the sweeps' own vectors (the blocks' stored residuals
                          and the half-spinors handed across block faces): QCD_F16 = FP16
                          with a power-of-two scale per site (per face entry), allowed with
                          F16/BF16 storage; any other value keeps the arithmetic precision.
                          The input and the output keep the arithmetic precision. */
} qcd_sap;

int sap_precond(qcd_field f, const qcd_sap *sap, const void *eta, void *psi, int nrhs, qcd_prec io,
                hipStream_t stream);

/* Block-local deflation (section 2.2): Ns global fields, drawn as complex
 * Gaussians from the counter-based generator SplitMix64 (key derived from
 * seed), refined by ninv rounds of the inverse iteration phi <- M_SAP phi
 * (normalised), restricted to the deflation blocks and orthonormalised per
 * block by two passes of modified Gram-Schmidt.  The little operator
 * A_kl = (phi_k, M phi_l) (eq. little) is assembled in FP64 with its
 * nearest-neighbour block structure, and its diagonal blocks are inverted.
 * Then nref further rounds of the inverse iteration phi <- M^{-1} phi
 * (normalised), each solve done by the deflated SAP-GCR solver on the
 * current subspace to relative residual ref_res (section 2.2: the inverse
 * iteration refined with the deflated solver), each round followed by a new
 * subspace and little operator.
 * The deflation block defaults to the Schwarz block (the paper ties the two
 * for simplicity); block[] may instead give a multiple of the Schwarz block
 * in every direction, with an even number of deflation blocks along each
 * axis (else QCD_EGEOM).  Ns > 12 x deflation-block volume: QCD_ESINGULAR. */
typedef struct {
    int Ns;
    int ninv;
    unsigned long long seed;
    qcd_sap sap;           /* preconditioner of the inverse iteration (and of the refinement solves) */
    int block[4];          /* deflation block (t, x, y, z); all 0: the Schwarz block */
    int nref;              /* rounds of inverse iteration with the deflated solver (0: none) */
    double ref_res;        /* relative residual of those solves, in (0, 1) */
} qcd_dfl_params;

int deflation_setup(qcd_field f, const qcd_dfl_params *p, hipStream_t stream, qcd_dfl *out);
int deflation_destroy(qcd_dfl d);
/* Deflation fields as complex128 DEVICE buffer [Nb][Ns][Vb][4][3]: deflation
 * block B in lexicographic order of the deflation-block grid, site j of the
 * block (Vb = deflation-block volume) in lexicographic order of local
 * coordinates. */
int deflation_get_phi(qcd_dfl d, void *phi, hipStream_t stream);
/* Replace the fields (same layout; must be block-orthonormal) and rebuild
 * the little operator; lets a caller supply a known basis. */
int deflation_set_phi(qcd_dfl d, const void *phi, hipStream_t stream);
/* Little-operator sizes: Nb blocks, Ns fields, N = Nb*Ns. */
int deflation_dims(qcd_dfl d, int *Nb, int *Ns);
/* w = A v for nrhs little vectors, complex128 DEVICE [nrhs][Nb][Ns] with the
 * block order of deflation_get_phi. */
int little_dirac_apply(qcd_dfl d, const void *v, void *w, int nrhs, hipStream_t stream);
/* w = A^{-1} v in FP64 by the block even-odd Schur complement (blocks
 * coloured by the parity of their coordinates on the deflation-block grid):
 * GCR on S = A_EE - A_EO A_OO^{-1} A_OE preconditioned with the inverse
 * diagonal blocks A_EE^{-1}, then x_O = A_OO^{-1} (v_O - A_OE x_E); to
 * relative residual ||v - A w|| / ||v|| <= tol (or maxit iterations); iters
 * (host, may be NULL) receives the iteration count. */
int little_dirac_solve(qcd_dfl d, const void *v, void *w, int nrhs, double tol, int maxit, int *iters,
                       hipStream_t stream);
/* Phi^+ v (restriction, complex128 [nrhs][Nb][Ns]) and Phi c
 * (prolongation, canonical vectors) for canonical io vectors. */
int deflation_restrict(qcd_dfl d, const void *v, void *u, int nrhs, qcd_prec io, hipStream_t stream);
int deflation_prolong(qcd_dfl d, const void *u, void *v, int nrhs, qcd_prec io, hipStream_t stream);

/* GCR solve of M x = b (section 2.2: right-preconditioned GCR on
 * D M_SAP phi = eta, psi = M_SAP phi), flexible, restarted.
 * The outer loop keeps x and the residual in FP64 and recomputes
 * r = b - M x with the FP64 operator at every restart; inside a cycle the
 * Krylov vectors are stored in FP32, the preconditioner runs at sap.storage
 * and the Gram-Schmidt coefficients are accumulated in FP64.
 * With a deflation handle the solution is psi = chi + Phi A^{-1} Phi^+ eta
 * (eq. deflsoln): GCR starts from the low-mode part and every search
 * direction is projected by P_R.
 * Stopping: relative residual ||b - M x||/||b|| <= res (FP64), or exactly
 * fixed_iters iterations when fixed_iters > 0 (truncated solves), or nmx. */
typedef struct {
    int nkv;            /* Krylov vectors per cycle */
    int nmx;            /* iteration limit */
    int fixed_iters;    /* > 0: stop after exactly this many iterations */
    double res;         /* target relative residual */
    qcd_sap sap;        /* preconditioner */
    qcd_dfl dfl;        /* NULL: no deflation */
    double little_tol;  /* relative residual of the little solves */
    int little_maxit;
} qcd_gcr;

typedef struct {
    int status;       /* 0 converged, QCD_NOCONV otherwise */
    int iters;
    double rel_res;   /* FP64 ||b - M x|| / ||b|| recomputed at exit */
} qcd_info;

int gcr_solve(qcd_field f, const qcd_gcr *p, const void *b, void *x, int nrhs, qcd_prec io,
              qcd_info *info /* host [nrhs] */, hipStream_t stream);

/* All-mode averaging (section 2.1).  The estimator
 *   O_AMA = (1/N_org) sum_{f in F} [O^f - O^(appx)f] + (1/N_G) sum_{g in G} O^(appx)g
 * (eqs. caa1, caa2) needs truncated ("sloppy") solutions for every source g
 * of the set G and exact ones for a subset F of G.  A source is one of:
 *   QCD_SRC_POINT  the 12 spin-colour point sources delta_{x,pos}
 *                  delta_{sc,sc'} (12 right-hand sides, sc = 3*spin+colour);
 *                  positions of one set must be related by translations of
 *                  whole blocks with an even total number of block steps, so
 *                  that M_SAP is covariant under them (section 2.2), else
 *                  QCD_EGEOM;
 *   QCD_SRC_Z2     nvec Z2-noise vectors, numbers index .. index+nvec-1 of
 *                  the stream `seed` (the vectors of make_z2_sources);
 *   QCD_SRC_SEQ    the 12 sequential sources (section 2.3) of 12 forward
 *                  solutions vec (DEVICE, canonical, io precision):
 *                  gamma_5 gamma_mu gamma_5 psi on timeslice t_sink, zero
 *                  elsewhere (as make_sequential_sources);
 *   QCD_SRC_VEC    nvec caller vectors vec (DEVICE, canonical, io precision).
 * Outputs: x_sloppy[i] receives the solutions of source i (all its vectors
 * in order, canonical, sloppy_out precision); x_exact[e] those of the e-th
 * source flagged in exact[] (io precision).  info_sloppy / info_exact (host,
 * may be NULL) get one entry per right-hand side in the same order.
 * Sloppy parameters with fixed_iters > 0 (the truncated solves of section
 * 3.5, Table 3) run without host synchronisation, each batch size replayed
 * from one captured HIP graph; a solution the fixed count leaves above
 * sloppy.res is solved again with the residual-stopping solver (its info
 * then counts both solves' iterations); sloppy.res = 0 keeps every
 * truncated solution as it is (the paper's fixed N_iter).  Other solves
 * stop at their res.
 * Source vectors and outputs must not overlap.  Returns QCD_NOCONV when a
 * solution misses its target; errors as for gcr_solve. */
typedef enum { QCD_SRC_POINT = 0, QCD_SRC_Z2 = 1, QCD_SRC_SEQ = 2, QCD_SRC_VEC = 3 } qcd_src_kind;

typedef struct {
    int kind;                  /* qcd_src_kind */
    int pos[4];                /* POINT: (t, x, y, z) */
    unsigned long long seed;   /* Z2: noise stream */
    long long index;           /* Z2: first noise vector */
    int nvec;                  /* Z2, VEC: number of vectors (POINT, SEQ: 12) */
    int t_sink, mu;            /* SEQ: insertion timeslice and direction */
    const void *vec;           /* SEQ: 12 forward solutions; VEC: nvec sources */
} qcd_source;

typedef struct {
    int nsrc;
    const qcd_source *src;         /* host [nsrc] */
    const unsigned char *exact;    /* host [nsrc] or NULL: nonzero = also solve exactly */
    qcd_gcr sloppy, exact_params;
    qcd_prec sloppy_out;           /* QCD_F64 or QCD_F32 */
    int batch;                     /* right-hand sides per solver launch (0: library choice, what 60% of
                                      the available memory holds, at most 48, a multiple of 12 or even);
                                      a request that 90% cannot hold falls back to that choice */
} qcd_ama;

int ama_solve(qcd_field f, const qcd_ama *a, void *const *x_sloppy, void *const *x_exact, qcd_prec io,
              qcd_info *info_sloppy, qcd_info *info_exact, hipStream_t stream);

/* The AMA sets of several gauge fields (the orbit G over an ensemble,
 * section 2.1) in one call: sets[k], x_sloppy[k], x_exact[k],
 * info_sloppy[k], info_exact[k] belong to fields[k], with the meaning of
 * ama_solve.  Every field's handle keeps its own block shape, deflation
 * subspace, launch choices and captured graphs (an autotuner sets them per
 * field beforehand).  All sets are validated before the first launch; the
 * fields are then solved in order on `stream`, each field's solver work
 * buffers (and captured graphs) released to the library's cache once its
 * set is done, so that the work buffers peak at what the largest field
 * needs.  All handles must live on the current device. */
int ama_solve_multi(int nfield, const qcd_field *fields, const qcd_ama *sets, void *const *const *x_sloppy,
                    void *const *const *x_exact, qcd_prec io, qcd_info *const *info_sloppy,
                    qcd_info *const *info_exact, hipStream_t stream);

/* The solve of gcr_solve for nrhs right-hand sides given one by one
 * (b[r], x[r]: caller-owned device pointers to canonical [V][4][3] vectors
 * at io precision), in batches of `batch` (0: 12).  With graph != 0 the
 * solve must have a fixed iteration count (p->fixed_iters > 0, the
 * truncated solves of section 3.5, Table 3): it then runs without host
 * synchronisation, and its launches for one batch size are captured once
 * into a HIP graph (on a stream the handle owns) and replayed for every
 * later batch of that size, on `stream`.  Little solves inside then run
 * a fixed budget: p->little_maxit iterations in P_R, and one cycle of
 * max(12, p->little_maxit) iterations in the low-mode correction.
 * info[r].rel_res is the FP64 relative residual after the fixed
 * iterations; status QCD_NOCONV if it is above p->res.  Graphs are kept in the handle until a workspace buffer
 * grows or the handle is destroyed.  Calls must not overlap in time with
 * other calls on the same handle. */
int gcr_solve_batched(qcd_field f, const qcd_gcr *p, const void *const *b, void *const *x, int nrhs, qcd_prec io,
                      int batch, int graph, qcd_info *info /* host [nrhs] */, hipStream_t stream);

/* Sources built on the device, canonical [n][V][4][3] at io precision.
 *
 * Z2 noise (stochastic sources for all-mode averaging, section 2.1): real
 * +-1 on every component; component j = 12 lex + spin-colour of noise
 * vector k = index0 + r takes the sign of the top bit of SplitMix64 output
 * 12 V k + j, SplitMix64 started at the state sm64(seed, 6) (output 6 of
 * the sequence started at `seed`).  out: caller-owned device buffer of n
 * vectors. */
int make_z2_sources(qcd_field f, unsigned long long seed, long long index0, int n, void *out, qcd_prec io,
                    hipStream_t stream);

/* Sequential sources (three-point functions, section 2.3): eta_r(x) =
 * delta_{t(x), t_sink} gamma_5 gamma_mu gamma_5 psi_r(x) for n forward
 * solutions psi (device, canonical), in the chiral basis of the operator.
 * psi and eta must not overlap.  Errors: mu outside 0..3 or t_sink outside
 * the lattice give QCD_EINVAL. */
int make_sequential_sources(qcd_field f, const void *psi, void *eta, int n, qcd_prec io, int t_sink, int mu,
                            hipStream_t stream);

/* Nucleon correlators from point-source propagators (section 2.3) and the
 * all-mode-averaging combination of observables (section 2.1).
 *
 * A propagator `prop` is the 12 canonical solutions x_j = M^{-1} b_j of the
 * point sources b_j = delta_{x,x0} e_j, j = 3 spin + colour, at io precision
 * (DEVICE, [12][V][4][3]); S(x)[s c][s' c'] = x_{3s'+c'}(x)[s c].  The
 * nucleon field is N_al = eps_abc (u_a^T C gamma_5 d_b) u_{c,al} (eq. Nop)
 * with C = gamma_0 gamma_2 in the operator's chiral basis and the conjugate
 * Nbar = eps (ubar (dbar C gamma_5 ubar^T)); u and d are degenerate (both
 * propagators are S) and no 2 kappa normalisation factor is applied.  All
 * arithmetic is FP64; timeslice sums are reduced in a fixed order.
 *
 * nucleon_2pt: corr (DEVICE complex128 [T][4][4]) receives the zero-momentum
 * two-point function G(t)_{al al'} = sum over the sites x of timeslice
 * (t0 + t) mod T of <N_al(x) Nbar_al'(x0)> by Wick's theorem
 *   eps_abc eps_a'b'c' [ S^{cc'} tr(Gamma S^{bb'} Gamma S^{aa' T})
 *                        - S^{ca'} (Gamma S^{bb'} Gamma)^T S^{ac'} ],
 * Gamma = C gamma_5; t0 is the source timeslice.  Projected correlators
 * tr(P G(t)) use P+ = (1 + gamma_0)/2 forward and P- backward.
 *
 * nucleon_seq_sources: the 12 sequential sources of a three-point function
 * with the nucleon sink on timeslice t_sink, zero momentum, projected with
 * the spin matrix proj (HOST complex128 [4][4], row-major), for the current
 * on the u line (flavour 0, both u lines) or the d line (flavour 1):
 * eta_j(x)_i = gamma_5,ii conj(K(x)_{ij}) on t_sink and 0 elsewhere, where
 * K = d tr(proj C(x)) / d S_flavour(x).  eta: DEVICE [12][V][4][3] at io
 * precision, must not overlap prop.  The solutions Sigma_j = M^{-1} eta_j
 * carry the sink back to every site (gamma_5-hermiticity); the forward and
 * backward nucleons of the paper take t_sink = t0 + t_s with P+ and
 * t0 - t_s with P-.
 *
 * nucleon_3pt: corr (DEVICE complex128 [T]) receives
 *   sum over y of timeslice (t0 + t) mod T of
 *   sum_j (gamma_5 Sigma_j(y))^+ (gamma_op x_j(y)),
 * the three-point function with the current gamma_op (HOST complex128
 * [4][4] spin matrix, identity in colour) inserted at time t, from the
 * sequential propagators seqprop = Sigma and the propagator prop.
 *
 * ama_combine: out[k] = (1/n_org) sum_f (exact_f[f][k] - appx_f[f][k])
 *   + (1/n_g) sum_g appx_g[g][k]   (eqs. caa1, caa2)
 * for DEVICE complex128 arrays appx_g [n_g][len], exact_f and appx_f
 * [n_org][len] (n_org may be 0), out [len]; observables of different
 * sources must already be aligned (e.g. time relative to each source).
 * Errors: null pointers, timeslices outside the lattice, bad flavour or
 * sizes give QCD_EINVAL. */
int nucleon_2pt(qcd_field f, const void *prop, qcd_prec io, int t0, void *corr, hipStream_t stream);
int nucleon_seq_sources(qcd_field f, const void *prop, qcd_prec io, int t_sink, const double *proj, int flavour,
                        void *eta, hipStream_t stream);
int nucleon_3pt(qcd_field f, const void *seqprop, const void *prop, qcd_prec io, int t0, const double *gamma_op,
                void *corr, hipStream_t stream);
int ama_combine(long long len, int n_g, const void *appx_g, int n_org, const void *exact_f, const void *appx_f,
                void *out, hipStream_t stream);

/* Source and sink smearing (section 2.3: Gaussian smearing with APE-smeared
 * gauge links in the Laplacian; the paper takes the parameters from earlier
 * work, so they are arguments here).
 *
 * qcd_field_ape_smear: n_iter APE steps of the handle's spatial links, kept
 * in the handle (FP64) for gauss_smear; time links are not smeared.  A step:
 *   U'_i(x) = P[(1 - alpha) U_i(x) + (alpha/4) sum_{j != i spatial}
 *             (U_j(x) U_i(x+j) U_j(x+i)^+ + U_j(x-j)^+ U_i(x-j) U_j(x-j+i))]
 * with P the projection onto SU(3): the unitary polar factor W of its
 * argument divided by exp(i arg(det W) / 3), arg in (-pi, pi].  n_iter = 0
 * keeps the unsmeared links.  Errors: QCD_EINVAL (n_iter < 0), QCD_ENOMEM.
 *
 * qcd_field_get_ape_links: the smeared links as DEVICE complex128
 * [V][3][3][3] (lexicographic site, direction i = mu - 1, row-major);
 * QCD_ENOTSET before qcd_field_ape_smear.
 *
 * gauss_smear: out = S^n_iter in for nrhs canonical vectors (io precision,
 * DEVICE; in and out may coincide), one step
 *   psi'(x) = [psi(x) + kappa_g sum_{i spatial} (U'_i(x) psi(x+i)
 *             + U'_i(x-i)^+ psi(x-i))] / (1 + 6 kappa_g),
 * colour only, each timeslice on its own, periodic in space, FP64
 * arithmetic.  QCD_ENOTSET before qcd_field_ape_smear. */
int qcd_field_ape_smear(qcd_field f, double alpha, int n_iter, hipStream_t stream);
int qcd_field_get_ape_links(qcd_field f, void *links, hipStream_t stream);
int gauss_smear(qcd_field f, const void *in, void *out, int nrhs, qcd_prec io, double kappa_g, int n_iter,
                hipStream_t stream);

/* Launch choices of a handle's Dirac stencil and Schwarz sweeps, for the
 * autotuner (defaults: block-staged, automatic, lexicographic, automatic,
 * 1, 1):
 * QCD_TUNE_STENCIL_BLOCK  1 = one workgroup per Schwarz block with the
 *                         block's spinors staged in LDS (when it fits),
 *                         0 = site tiles;
 * QCD_TUNE_STENCIL_RG     right-hand sides per site tile: 0 (automatic),
 *                         1, 2 or 4;
 * QCD_TUNE_STENCIL_ORDER  1 = site tiles in lexicographic block order,
 *                         0 = memory order;
 * QCD_TUNE_STENCIL_NR     block-staged kernel: right-hand sides per
 *                         workgroup, sharing each link and clover load:
 *                         0 (automatic: 2), 1, 2 or 4; reduced to a divisor
 *                         of the call's count whose staged blocks fit the
 *                         device's LDS per workgroup (FP16 spinors: 1);
 * QCD_TUNE_STENCIL_LINKLDS FP32 vectors with FP16/BF16 links, at least 16
 *                         right-hand sides, blocks of at most 256 sites:
 *                         1 = one workgroup per block keeps the block's
 *                         links in LDS and loops over the right-hand sides
 *                         two at a time, 0 = the block-staged kernel above;
 * QCD_TUNE_SAP_PAIR       Schwarz sweeps with FP32 arithmetic on blocks of
 *                         128 sites per parity (4^4) and an even number of
 *                         right-hand sides: 1 = two right-hand sides per
 *                         workgroup, sharing link and clover loads (the
 *                         block reductions then add in another order), 0 =
 *                         one.
 * Results do not depend on these beyond rounding; graphs captured on the
 * handle are dropped.  Unknown knob or value: QCD_EINVAL. */
#define QCD_TUNE_STENCIL_BLOCK 0
#define QCD_TUNE_STENCIL_RG 1
#define QCD_TUNE_STENCIL_ORDER 2
#define QCD_TUNE_STENCIL_NR 3
#define QCD_TUNE_STENCIL_LINKLDS 4
#define QCD_TUNE_SAP_PAIR 5
int qcd_field_tune(qcd_field f, int knob, int value);

/* Process-wide workspace cache.  Scratch buffers that a handle gives up
 * (outgrown, or the handle destroyed) are kept for later handles on the
 * same device; a cached buffer serves requests of half its size up to its
 * size.  qcd_workspace_cached stores in *bytes what the cache holds for a
 * device (memory that the device's free-memory query counts as used);
 * qcd_workspace_trim frees it (device < 0: every device), waiting for the
 * device first.  Buffers held by live handles are not touched.  Neither
 * call may overlap a call that uses the workspace.  Null bytes: QCD_EINVAL. */
int qcd_workspace_cached(int device, size_t *bytes);
int qcd_workspace_trim(int device);
/* Hand a handle's scratch buffers back to the workspace cache (after its
 * queued work is done), so that another handle of the same lattice reuses
 * them; the handle allocates again on its next call, and its captured
 * graphs are dropped.  Null handle: QCD_EINVAL. */
int qcd_field_trim(qcd_field f);

/* Kernel timing with HIP events on the launch stream, for measurement.
 * Classes: 0 Dirac stencil, 1 SAP block sweep, 2 deflation projection and
 * prolongation, 3 little operator, 4 vector algebra, 5 other. */
#define QCD_PROF_CLASSES 6
int qcd_prof_enable(int on);
int qcd_prof_reset(void);
/* Total milliseconds and launch count for a class since the last reset
 * (synchronises the recorded events). */
int qcd_prof_get(int cls, double *ms, long long *launches);
/* Algorithmic work of the recorded launches of a class: flops, compulsory
 * HBM bytes and work units (site applications per right-hand side; for the
 * SAP class one unit is one site visited by one colour sweep).  The per-unit
 * figures are: stencil 1872 flop; SAP sweep see sap.hip; vector algebra 0. */
int qcd_prof_get_work(int cls, double *flops, double *bytes, double *units);

#ifdef __cplusplus
}
#endif
#endif
