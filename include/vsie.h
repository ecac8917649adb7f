/*
 * vsie.h -- C ABI of the MI355X hybrid volume-surface integral equation (VSIE) library.
 *
 * The library builds and applies the hybrid VSIE operator of Giannakopoulos et al.,
 * "A hybrid volume-surface integral equation method for rapid electromagnetic simulations in
 * MRI" (arXiv 2206.12409), Sec. III eq. (15):
 *
 *     [ Z_cc^ff        conj(V) U^T    Zt^T          ] [ j_far  ]   [ v_far  ]
 *     [ U V^*          Z^pFFT (near, body)          ] [ j_near ] = [ v_near ]
 *     [ Zt             (eq. (13))                   ] [ j_body ]   [ 0      ]
 *
 * where Z_cc^ff is the dense Galerkin matrix of the far conductors (eq. (6)), U V^* the adaptive
 * cross approximation of the near-far conductor block (eq. (12)), Zt the tensor-train
 * compressed far coupling (eq. (14)), and Z^pFFT the precorrected-FFT operator of the near
 * conductors and the voxelised body (eq. (13)) whose volume part is the block-Toeplitz
 * convolution of Sec. II-B.
 *
 * Conventions (fixed by the paper's statement of the problem, Sec. II):
 *   - exp(+i w t) time dependence; g(R) = exp(-i k0 R) / (4 pi R);
 *   - complex susceptibility chi = eps_r - 1 - i sigma / (w eps0); voxels with chi = 0 are air
 *     and carry identity rows and columns;
 *   - every row multiplied by i w eps0; body rows tested with the field (eq. (4) divided by chi),
 *     so the matrix is complex symmetric (eq. (8));
 *   - unknown vector, complex interleaved, length N = m_f + m_n + 3 n_v:
 *         [ j_far (m_f) | j_near (m_n) | j_body^x (n_v) | j_body^y (n_v) | j_body^z (n_v) ]
 *     far and near RWG functions in mesh input order, edges of a mesh sorted by
 *     (min vertex, max vertex); voxels with i1 fastest, flat index i1 + n1 (i2 + n2 i3);
 *   - RWG orientation: for edge (a, b), a < b, T+ is the triangle listing a then b in cyclic
 *     order; positive current flows from T+ into T-.
 *
 * Error convention: every call returns an int status (VSIE_OK = 0). On failure a thread-local
 * message is available from vsie_last_error(). Nothing throws across this interface.
 * Streams are hipStream_t passed as void* (NULL = the default stream).
 */
#ifndef VSIE_H
#define VSIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum vsie_status {
  VSIE_OK = 0,
  VSIE_E_ARG = 1,          /* null pointer, bad size, non-finite value */
  VSIE_E_MESH = 2,         /* degenerate triangle, inconsistent orientation, bad port edge */
  VSIE_E_STENCIL = 3,      /* a near RWG pair does not fit its 5x5x5 expansion block (Sec. IV-B) */
  VSIE_E_GRID = 4,         /* grid or extended grid too large */
  VSIE_E_NOMEM = 5,        /* device or host allocation failed */
  VSIE_E_HIP = 6,          /* a HIP runtime call failed */
  VSIE_E_NOCONV = 7,       /* solver hit max_iter; statistics are still filled */
  VSIE_E_BREAKDOWN = 8,    /* Arnoldi breakdown without convergence */
  VSIE_E_UNSUPPORTED = 9,  /* option not supported (e.g. piecewise-linear basis) */
  VSIE_E_STATE = 10,       /* operation not valid for this handle (e.g. precision not built) */
  VSIE_E_SINGULAR = 11     /* dense factorisation met an exactly zero pivot column */
};

enum vsie_domain { VSIE_NEAR = 0, VSIE_FAR = 1 };
enum vsie_dtype { VSIE_C128 = 0, VSIE_C64 = 1 };
/* basis of the body currents (Sec. II-B): piecewise constant (3 unknowns per voxel) or piecewise
 * linear (12 per voxel; not built, vsie_create returns E_UNSUPPORTED) */
enum vsie_basis { VSIE_BASIS_PWC = 0, VSIE_BASIS_PWL = 1 };
/* operator data held by the handle: complex128 only, or complex128 plus complex64 copies for the
 * complex64 product and the mixed-precision solvers */
enum vsie_precision { VSIE_PREC_FP64 = 0, VSIE_PREC_MIXED = 1 };

/* A triangle mesh of a perfectly conducting surface (Sec. II-B, RWG basis). */
typedef struct {
  const double* verts;        /* [n_verts][3] metres, host memory, copied by vsie_create */
  int32_t n_verts;
  const int32_t* tris;        /* [n_tris][3] vertex ids, consistently oriented */
  int32_t n_tris;
  int32_t domain;             /* VSIE_NEAR (pFFT, Sec. III) or VSIE_FAR (TT + ACA + dense) */
  const int32_t* port_edges;  /* [n_port_edges][2] directed interior edges (a, b); may be NULL */
  const int32_t* port_id;     /* [n_port_edges] port number within this mesh, 0..n_ports-1 */
  int32_t n_port_edges;
} vsie_mesh;

/* The voxelised body and the conductors (Sec. II-B, Sec. IV-A/B). */
typedef struct {
  int32_t n[3];               /* voxels per axis */
  double h;                   /* voxel edge, metres */
  double origin[3];           /* lower corner of voxel (0,0,0) */
  double freq_hz;             /* operating (Larmor) frequency */
  const double* eps_r;        /* [n3][n2][n1] relative permittivity, host */
  const double* sigma;        /* [n3][n2][n1] conductivity S/m, host */
  int32_t n_meshes;
  const vsie_mesh* meshes;
} vsie_problem;

/* Setup options. The discretisation fields fix the operator the paper defines (Sec. II-B, Sec. IV-B,
 * Sec. IV-C); values other than the listed ones give E_UNSUPPORTED. */
typedef struct {
  double tt_tol;              /* TT-cross relative accuracy, Sec. IV-C: 1e-3 */
  int32_t tt_rank_max;        /* rank cap per TT unfolding, 1..128 */
  double aca_tol;             /* ACA relative accuracy, Sec. IV-C: 1e-3 */
  int32_t aca_rank_max;       /* 1..256 */
  int32_t precorrect_dist;    /* Chebyshev distance (voxels) of precorrected pairs, default 2 */
  int32_t precision;          /* VSIE_PREC_FP64 or VSIE_PREC_MIXED (default) */
  int32_t build_far;          /* compute TT-cross and ACA (0: zero far coupling until imported) */
  uint64_t seed;              /* TT-cross initial index sets, ACA held-out rows */
  int32_t basis;              /* VSIE_BASIS_PWC (default); VSIE_BASIS_PWL: E_UNSUPPORTED */
  int32_t stencil;            /* pFFT expansion block edge in voxels, Sec. IV-B: 5 */
  int32_t quad_near_vol;      /* near coupling, volume points per voxel, Sec. IV-C: 8 (2x2x2 Gauss) */
  int32_t quad_near_surf;     /* near coupling, points per triangle: 5 */
  int32_t quad_far_vol;       /* far coupling (TT-cross entries): 1 (voxel centre) */
  int32_t quad_far_surf;      /* far coupling: 1 (triangle centroid) */
} vsie_options;

typedef struct {
  int64_t n_total;            /* N */
  int32_t m_far, m_near;      /* RWG counts */
  int32_t n[3];               /* body grid */
  int32_t n_ext[3];           /* extended (pFFT) grid enclosing body and near stencils */
  int32_t fft[3];             /* circulant FFT size per axis */
  int32_t n_ports;
  int32_t n_tissue;           /* voxels with chi != 0 */
  int32_t tt_rank[3][3];      /* [component][unfolding] */
  double tt_err_est[3];       /* held-out relative error estimate of each TT */
  int32_t aca_rank;
  int64_t precorr_nnz;
  int64_t device_bytes;       /* operator data held on the device */
  double setup_seconds;
} vsie_sizes_t;

typedef struct {
  double tol;                 /* relative residual ||b - Ax|| / ||b||, default 1e-6 */
  int32_t restart;            /* GMRES restart length, default 50 (Sec. IV-C) */
  int32_t max_iter;           /* GMRES64: iterations; IR_MIXED: total inner complex64 iterations */
  int32_t method;             /* a vsie_method */
  double inner_tol;           /* IR_MIXED: inner complex64 solve tolerance, default 1e-3 */
  int32_t precond;            /* SCHUR: 1 (default) right-preconditions the reduced system, 0 none */
  double reorth;              /* Gram-Schmidt: a second classical pass follows a first that leaves less
                                 than this fraction of the new vector's norm (the test of Daniel, Gragg,
                                 Kaufman and Stewart, whose classical constant is 1/sqrt(2)); default
                                 0.1, which bounds the orthogonality lost by a single pass at about
                                 ten roundings; 0 = always one pass; must lie in [0, 1] (else E_ARG) */
} vsie_solve_opts;

enum vsie_method {
  VSIE_GMRES64 = 0,
  VSIE_IR_MIXED = 1,
  VSIE_SCHUR = 2,
  VSIE_SCHUR_MIXED = 3,
  VSIE_SCHUR_LEARNED = 4   /* reduced system, flexible GMRES with the attached network (vsie_net_attach) */
};

typedef struct {
  int32_t iterations;         /* Krylov iterations (IR_MIXED: inner complex64 iterations) */
  int32_t restarts;
  int32_t refinements;        /* IR_MIXED: FP64 outer steps, one FP64 product and inner solve each */
  double rel_residual;        /* true FP64 ||b - Ax|| / ||b|| at exit */
  double block_residual[3];   /* relative residual restricted to far / near / body rows */
  double seconds;
  int32_t gs_second_passes;   /* Arnoldi steps that took the second Gram-Schmidt pass */
} vsie_solve_stats;

/* Fill defaults: tt_tol 1e-3, tt_rank_max 96, aca_tol 1e-3, aca_rank_max 256,
 * precorrect_dist 2, precision VSIE_PREC_MIXED, build_far 1, seed 1, basis VSIE_BASIS_PWC,
 * stencil 5, quadrature 8 / 5 near and 1 / 1 far. */
int vsie_default_options(vsie_options* opts);
int vsie_default_solve_opts(vsie_solve_opts* opts);

/* Set up the operator (Sec. III): RWG tables, extended grid, Green-tensor generator and its
 * circulant spectra (Sec. II-B), pFFT stencils and precorrection (eq. (13)), TT-cross of the far
 * coupling (eq. (14)), ACA of the near-far block (eq. (12)), dense Z_cc^ff (eq. (6)).
 * All inputs are copied; the handle owns every device allocation (the dense far block may be
 * shared with handles made by vsie_create_shared). Blocks until done.
 * Errors: E_ARG, E_MESH, E_STENCIL, E_GRID, E_NOMEM, E_HIP, E_UNSUPPORTED. */
int vsie_create(const vsie_problem* problem, const vsie_options* opts, void* stream,
                struct vsie_handle** out);

/* As vsie_create, but the dense far block Z_cc^ff (eq. (6)) and its tiling are taken from donor
 * instead of assembled: for several phantoms inside the same far conductors (shield) at the same
 * frequency. The far meshes (vertices, triangles and their order, hence the RWG numbering) and the
 * frequency must equal the donor's, else E_ARG. The block is shared, not copied: it stays allocated
 * while any handle built on it lives, in any destruction order; the complex64 copy is shared too.
 * Errors: as vsie_create; E_STATE when the donor has no dense far block. */
int vsie_create_shared(const vsie_problem* problem, const vsie_options* opts, struct vsie_handle* donor,
                       void* stream, struct vsie_handle** out);

/* Sizes of the discrete system of eq. (15) (unknown counts of Sec. III: far and near RWG functions,
 * three PWC components per voxel), the extended pFFT grid and its circulant FFT sizes (Sec. II-B),
 * the compression ranks (eqs. (12), (14)), device bytes and setup time. Host only. Errors: E_ARG. */
int vsie_sizes(const struct vsie_handle* h, vsie_sizes_t* out);

/* Delta-gap right-hand side of one port (Sec. II-A after eq. (2)): b_m = s_m i w eps0 V0 l_m,
 * V0 = 1 V, into the caller-owned device buffer b_dev of N complex values of type dtype. The port
 * tables live on the device from vsie_create on: this call only launches a fill and a scatter on
 * the stream (asynchronous, no allocation, no synchronisation). Errors: E_ARG (port out of range,
 * bad dtype, null pointer). */
int vsie_rhs(const struct vsie_handle* h, int port, int dtype, void* b_dev, void* stream);

/* y = Z x, the hybrid operator of eq. (15) (far block eq. (6), ACA block eq. (12), pFFT block
 * eq. (13) with the block-Toeplitz volume convolution of Sec. II-B, TT coupling eqs. (16)-(19)), for
 * nrhs columns, layout [nrhs][N] complex interleaved (complex128 or complex64 as dtype says),
 * device memory owned by the caller, 256-byte aligned, x and y must not alias.
 * Asynchronous on stream. The handle's work buffers serialise calls on one handle.
 * Errors: E_ARG, E_STATE (complex64 data not built), E_HIP. */
int vsie_matvec(struct vsie_handle* h, int dtype, int nrhs, const void* x_dev, void* y_dev,
                void* stream);

/* The same product as vsie_matvec, with the same result bit for bit, replayed from a HIP graph:
 * the first call with a given (dtype, nrhs, x_dev, y_dev) waits for stream, captures the
 * product's launches on the handle's capture stream and instantiates them; every call then launches
 * the graph on stream (one submission instead of one per kernel). The graph holds the buffer
 * addresses: they must stay allocated, with nrhs N elements each, while the handle may replay it.
 * Up to 16 graphs are kept per handle (the oldest is dropped). Errors: as vsie_matvec. */
int vsie_matvec_graph(struct vsie_handle* h, int dtype, int nrhs, const void* x_dev, void* y_dev,
                      void* stream);

/* Products of several operators in one launch: one HIP graph holding, one operator after another,
 * the launches of vsie_matvec(hs[i], dtype, nrhs[i], x[i], y[i]) for i < n (phantoms of different
 * grids and ports in one batch, e.g. inside one shield); vsie_graph_launch replays all of them on
 * stream, with the results of n separate vsie_matvec calls bit for bit. The operators and buffers
 * must outlive the graph, and an operator may appear only once (its work buffers serve one product
 * at a time); creation waits for stream. Errors: E_ARG, E_STATE (complex64 data not built), E_HIP,
 * E_NOMEM. */
typedef struct vsie_graph vsie_graph;
int vsie_graph_create(int n, struct vsie_handle* const* hs, int dtype, const int* nrhs,
                      const void* const* x_dev, void* const* y_dev, void* stream, vsie_graph** out);
int vsie_graph_launch(vsie_graph* g, void* stream);
int vsie_graph_destroy(vsie_graph* g);

/* The z pass of the block-Toeplitz convolution (Sec. II-B: the FFT along the third axis with the
 * 3 x 3 spectral product) is compiled in up to three radix/tile candidates per FFT length:
 * 0 the default, 1 half the pencils per workgroup, 2 twice the values per thread. vsie_create
 * times each candidate on the operator's own buffers (three launches after a warm-up) and keeps the
 * fastest, per precision. vsie_zpass_tuning reports, for dtype (VSIE_C128 / VSIE_C64): the chosen
 * candidate, and per candidate c < 3 its values per thread v[c], pencils per workgroup np[c] and
 * measured milliseconds per launch ms[c] (v[c] = np[c] = 0 and ms[c] = 0 where a candidate does not
 * exist for this length; all zero for FFT lengths outside 64..1024). vsie_zpass_select makes
 * candidate cand the one in use (for tests and experiments; cached graphs are dropped).
 * Errors: E_ARG, E_STATE (complex64 data not built; no candidates for this grid). */
int vsie_zpass_tuning(struct vsie_handle* h, int dtype, int* chosen, int* v, int* np, double* ms);
int vsie_zpass_select(struct vsie_handle* h, int dtype, int cand);

/* Solve Z x = b for nrhs right-hand sides (device, [nrhs][N] complex128).
 * GMRES64: restarted GMRES (Sec. III-A), zero initial guess, FP64 classical Gram-Schmidt with a
 * second pass when the first leaves less than opts->reorth of the new vector's norm.
 * IR_MIXED: FP64 flexible GMRES (20 steps per cycle) on the FP64 operator whose preconditioner is
 * one cycle (at most `restart` iterations, stopping early at inner_tol) of complex64 GMRES on
 * Z z = v; with an exact inner solve each outer step is one refinement x += Z^{-1}(b - Zx).
 * SCHUR: the far-conductor currents are eliminated first (see vsie_schur_setup) and FP64 GMRES
 * runs on the reduced system (near currents and body) with zero initial guess, right-preconditioned
 * by the block-diagonal operator of vsie_schur_precond; the far currents are recovered afterwards.
 * The residual test is on the full system's relative residual.
 * SCHUR_MIXED: the same reduced, preconditioned system solved as IR_MIXED does: FP64 flexible
 * GMRES (20 steps per cycle) whose preconditioner is one complex64 GMRES cycle on the complex64
 * reduced operator (iterations count the inner ones, refinements the FP64 steps).
 * SCHUR_LEARNED: FP64 flexible GMRES (restart `restart`) on the reduced system with the variable
 * right preconditioner P(v) = M v + (learned body correction of the attached network, see
 * vsie_net_attach); iterations count the preconditioner applications, refinements the flexible
 * steps. Needs an attached network (else E_STATE); builds the SCHUR preconditioner M.
 * x_dev receives complex128. Blocks.
 * The Krylov basis and work vectors hold only the unknowns that couple (far and near currents,
 * tissue voxels): air voxels carry identity rows and columns, so their solution is b there.
 * Allocates its work vectors (IR_MIXED: 41 FP64 vectors of that length besides the basis).
 * stats (array of nrhs, may be NULL) are filled even on E_NOCONV. */
int vsie_solve(struct vsie_handle* h, const vsie_solve_opts* opts, int nrhs, const void* b_dev,
               void* x_dev, vsie_solve_stats* stats, void* stream);

/* The coil-port solves of the paper (one GMRES solve per channel, Sec. IV-C; Table I averages the
 * channels): for each of the nports port numbers in ports (host array) the delta-gap right-hand
 * side of vsie_rhs is formed on the device and Z x = b is solved as vsie_solve does with the same
 * options; x_dev ([nports][N] complex128, caller-owned device memory) receives the solutions and
 * stats (may be NULL) one entry per port. Blocks. Allocates the right-hand sides besides
 * vsie_solve's work vectors. Errors: E_ARG (null pointer, nports < 1, port out of range), and
 * those of vsie_solve. */
int vsie_solve_ports(struct vsie_handle* h, const vsie_solve_opts* opts, int nports, const int32_t* ports,
                     void* x_dev, vsie_solve_stats* stats, void* stream);

/* Port current I = sum_m s_m l_m x_m of a solution held in host memory (complex128, length N):
 * the current through the delta-gap edge of Sec. II-A; the input admittance is I / V0, V0 = 1 V. */
int vsie_port_current(const struct vsie_handle* h, int port, const double* x_host, double* I_re_im);

/* Setup artefacts (host copies): the compressed blocks that Sec. VI proposes to store and recycle
 * (TT cores of eq. (14), ACA factors of eq. (12)), the pFFT stencils of eq. (13) and the Toeplitz
 * generator of Sec. II-B, for checkpointing and for tests. `index` selects the TT
 * component (0..2) where relevant. Call with host == NULL to query the byte count.
 *   VSIE_X_TT_CORES    int32 r1,r2,r3 then complex128 G1[n1][r1], G2[r1][n2][r2],
 *                      G3[r2][n3][r3], G4[r3][m_f]
 *   VSIE_X_ACA         int32 k then complex128 U[m_n][k], V[m_f][k]  (Z_nf ~ U V^*), k <= 256
 *   (TT ranks accepted by vsie_import: 1..128)
 *   VSIE_X_STENCIL     int32 base[m_n][3] (relative to the body grid) then double W[m_n][3][125]
 *   VSIE_X_GENERATOR   complex128 T[6][ne3][ne2][ne1] dimensionless generator on the octant
 *   VSIE_X_EXT_GRID    int32 ne[3], body_offset[3], fft[3] */
enum vsie_export_kind {
  VSIE_X_TT_CORES = 1,
  VSIE_X_ACA = 2,
  VSIE_X_STENCIL = 3,
  VSIE_X_GENERATOR = 4,
  VSIE_X_EXT_GRID = 5
};
int vsie_export(const struct vsie_handle* h, int what, int index, void* host, size_t* nbytes);

/* Replace a compressed block with stored data (the "store and recycle" use of the compressed
 * coupling, Sec. VI): VSIE_X_TT_CORES (one component per call) or VSIE_X_ACA, same layout as
 * vsie_export. Errors: E_ARG (size mismatch), E_STATE (after vsie_schur_setup, whose matrices
 * were formed from the factors in place). */
int vsie_import(struct vsie_handle* h, int what, int index, const void* host, size_t nbytes);

/* Persistent checkpoint of the setup products that cost the most to recompute: the TT cores of
 * the three far-coupling components (eq. (14)) and the ACA factors of the near-far block
 * (eq. (12)), the compressed coupling that Sec. VI proposes to store and reuse. Dense blocks,
 * stencils and spectra are not stored: they are rebuilt by vsie_create in seconds.
 *
 * File layout (host byte order): char[8] "VSIECKPT", uint32 version (1), uint64 key, uint32
 * record count, then per record uint32 kind (VSIE_X_TT_CORES or VSIE_X_ACA), uint32 index,
 * uint64 byte count and that many bytes in the vsie_export layout. The key is a 64-bit FNV-1a
 * hash of the inputs that fix the factors: grid sizes, spacing and origin, frequency, eps_r and
 * sigma, every mesh with its ports, and the options tt_tol, tt_rank_max, aca_tol, aca_rank_max,
 * seed, quad_far_vol and quad_far_surf.
 *
 * vsie_checkpoint_save writes path + ".part" and renames it to path, so a reader never sees a
 * partial file. Errors: E_ARG (null argument, file not writable), E_STATE (no far conductors).
 * vsie_checkpoint_load reads every record, then imports them as vsie_import does; intended for a
 * handle created with build_far = 0 from the same inputs. Products afterwards are bitwise equal
 * to those of the handle that saved the file. Errors: E_ARG (unreadable or damaged file, other
 * version, key differs from this handle's inputs: nothing is changed then), E_STATE (after
 * vsie_schur_setup). */
int vsie_checkpoint_save(const struct vsie_handle* h, const char* path);
int vsie_checkpoint_load(struct vsie_handle* h, const char* path);

/* Concurrency of one product: enable != 0 runs the far-block chain (gemv_far, gemv_far_reduce,
 * tt_pre: the dense far block and the TT stages that read only x) on a second non-blocking stream
 * of default priority, forked from and joined back into the caller's stream with events, while the
 * volume/pFFT chain runs on the caller's stream; 0 (the default) runs every stage in order on the
 * caller's stream. Results are identical either way. Waits for the second stream before it
 * returns. Errors: E_ARG, E_HIP. */
int vsie_set_concurrency(struct vsie_handle* h, int enable);

/* Per-stage timing of vsie_matvec with HIP events recorded on the stream each stage runs on.
 * vsie_profile_mask(h, stages) times the stages whose bit (1 << stage index) is set and resets the
 * totals (0 turns profiling off); vsie_profile(h, enable) is the same with all stages or none.
 * Event creation happens on first use. The events of up to 256 products are kept and read back by
 * vsie_profile_read (which waits for them) or when that ring is full, so products are not
 * synchronised while profiled. Stage indices: 0 build_grid, 1 fft_x_fwd, 2 fft_y_fwd,
 * 3 fft_z_conv, 4 fft_y_inv, 5 fft_x_inv, 6 body_out, 7 pfft_gather, 8 gemv_far, 9 precorrect,
 * 10 aca, 11 tt_pre, 12 gemv_far_reduce, 13 tt_post. vsie_profile_read returns up to max_stages
 * entries (names are static strings), the summed milliseconds and the number of timed calls per
 * stage, and the stage count. */
int vsie_profile(struct vsie_handle* h, int enable);
int vsie_profile_mask(struct vsie_handle* h, uint32_t stages);
int vsie_profile_read(const struct vsie_handle* h, int max_stages, const char** names, double* total_ms,
                      int64_t* calls, int* n_stages);

/* Elimination of the far-conductor currents (the Schur complement of the dense far block; the
 * paper's conclusion proposes solving for the other unknowns first). The far conductor couples to
 * the rest only through the ACA factors (eq. (12)) and the TT cores (eq. (14)), so with
 * L = [conj(V) | G4^T of each component] (m_f x K, K = ACA rank + the three TT ranks r3) the
 * reduced operator on the near currents and the body is
 *     A_S = Z_rr - Z_rf Z_ff^-1 Z_fr = Z_rr - R^T (L^T Z_ff^-1 L) R,
 * R the maps of eqs. (12) and (18)-(19) from x_r to the K proxies. vsie_schur_setup unpacks the
 * dense far block (m_f^2 complex128 held on the device), factors it (vsie_dense_lu_solve's
 * method), forms W = Z_ff^-1 L and the K x K matrix L^T W. With precond != 0 it also builds the
 * right preconditioner of vsie_schur_precond: the inverse of the reduced near block
 * (direct Galerkin entries of the near coils minus U (L^T W)_aa U^T; m_n^2 complex128 while
 * building) and the inverse body diagonal (h^3 / chi + h^3 T_aa(0)). Blocks; later calls only
 * add what is missing. Errors: E_NOMEM, E_SINGULAR, E_HIP, E_ARG (K > 640). */
int vsie_schur_setup(struct vsie_handle* h, int precond);
/* K (0 before setup or without far conductors), setup seconds so far, and whether the
 * elimination (bit 0) and the preconditioner (bit 1) are built. */
int vsie_schur_info(const struct vsie_handle* h, int32_t* n_proxy, double* seconds, int32_t* built);
/* y = A_S x on device vectors of length N (complex128, layout as vsie_matvec): the far part of x
 * is not read and the far part of y is set to zero. Asynchronous. Errors: E_STATE (no setup). */
int vsie_schur_matvec(struct vsie_handle* h, const void* x_dev, void* y_dev, void* stream);
/* y = M x, M = block diagonal: inverse reduced near block on the near currents, inverse body
 * diagonal on the body (1 on air voxels), zero on the far currents. Asynchronous.
 * Errors: E_STATE (preconditioner not built). */
int vsie_schur_precond(struct vsie_handle* h, const void* x_dev, void* y_dev, void* stream);

/* Dense complex128 solve A X = B on the device, row-major, A (n x n, row stride lda >= n)
 * overwritten by its LU factors (P A = L U, partial pivoting by |re| + |im|), B (n x nrhs, row
 * stride ldb >= nrhs) overwritten by X. Blocked right-looking factorisation with panels of 64
 * columns whose trailing updates run on the matrix cores. Caller-owned buffers; allocates its
 * scratch; blocks. Errors: E_ARG, E_SINGULAR (exactly zero pivot column), E_NOMEM, E_HIP. */
int vsie_dense_lu_solve(int n, void* A_dev, int64_t lda, void* B_dev, int64_t ldb, int nrhs, void* stream);

/* vsie_dense_lu_solve for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc). Same arguments, same kernels and
 * the same result; the workspace (inverted diagonal blocks, panel work, the n x nrhs solve buffer,
 * pivots, permutation, singularity flag) is a static device array of the library, about 16.8 MB,
 * held on every GPU the library runs on until the process ends; its address on a device is looked
 * up on the first call there. Sizes: n <= VSIE_LU_NOALLOC_MAX_N, nrhs <= VSIE_LU_NOALLOC_MAX_NRHS,
 * else E_ARG. Calls no hipMalloc, hipFree or other allocating routine, on the device or the host
 * (the row permutation is formed on the device; only the singularity flag is read back). Every
 * call on one GPU shares that GPU's workspace, which keeps the last call's contents: calls that
 * overlap on one GPU (several streams or host threads) race and must be serialised by the caller.
 * Blocks. Errors: E_ARG, E_SINGULAR, E_HIP. */
#define VSIE_LU_NOALLOC_MAX_N 4096
#define VSIE_LU_NOALLOC_MAX_NRHS 64
int vsie_dense_lu_solve_noalloc(int n, void* A_dev, int64_t lda, void* B_dev, int64_t ldb, int nrhs, void* stream);

/* ---------------------------------------------------------------------------------------------
 * Learned preconditioner (an addition to the paper's method, whose conclusion, Sec. VI, names a
 * Calderon preconditioner as future work). A 3D convolutional U-Net on the voxel grid (4 levels,
 * 16 to 64 channels, 3x3x3 convolutions, average pooling, nearest upsampling, ReLU; bfloat16
 * matrix-core convolutions with float32 accumulation, float32 master weights, Adam) maps the body
 * part of a residual (Re, Im of three components, scaled to unit RMS, plus two channels of the
 * body diagonal's inverse) to a correction of the body currents. Parameter layout (float32, the
 * order of the network's twelve layers e1a e1b e2a e2b e3a e3b e4a e4b d3 d2 d1 out): per layer
 * the weights [Cout][3][3][3][Cin] (taps z, y, x), then the biases [Cout].
 * The network object is independent of any handle: it collects training pairs from the solves of
 * one or several handles (phantoms) whose body grids agree, trains on them, and is attached to the
 * handle whose solves it preconditions. The network grid is the body grid rounded up to multiples
 * of 8 per axis. */
struct vsie_net;
/* New network: He-normal weights from a seeded generator, zero biases; room for pair_capacity
 * training pairs (bfloat16, 32 bytes per grid voxel each, allocated at the first collected pair).
 * Errors: E_ARG, E_NOMEM. */
int vsie_net_create(uint64_t seed, int64_t pair_capacity, struct vsie_net** out);
void vsie_net_destroy(struct vsie_net* net);
/* Parameter count, collected pairs and Adam steps taken (each pointer may be NULL). */
int vsie_net_info(const struct vsie_net* net, int64_t* nparam, int64_t* n_pairs, int64_t* adam_steps);
/* Copy the float32 parameters (layout above) to or from host memory; count must equal nparam.
 * Blocks. Errors: E_ARG. */
int vsie_net_get_params(const struct vsie_net* net, float* host, int64_t count);
int vsie_net_set_params(struct vsie_net* net, const float* host, int64_t count);
/* Training pairs from the preconditioned SCHUR solves of the given ports of h (opts->method must be
 * VSIE_SCHUR with precond 1): every Arnoldi step applies the reduced operator A_S to z = M v and
 * stores (input: body part of w = A_S z scaled to unit RMS with the material channels; target:
 * body part of z - D^-1 w over the same scale times the largest |D^-1|), until the capacity is
 * reached. *n_pairs receives the total held. Blocks. Errors: those of vsie_solve_ports except
 * E_NOCONV, E_ARG (grid differs from the pairs already held). */
int vsie_net_collect(struct vsie_net* net, struct vsie_handle* h, int nports, const int32_t* ports,
                     const vsie_solve_opts* opts, int64_t* n_pairs, void* stream);
/* epochs passes of Adam (learning rate lr, betas 0.9 / 0.999, eps 1e-8) over the stored pairs,
 * one pair per step in a seeded shuffled order, each pair under a random common complex phase;
 * loss = sum (y - t)^2 / (2 n); *last_loss = mean loss of the last epoch. Blocks.
 * Errors: E_ARG, E_STATE (no pairs). */
int vsie_net_train(struct vsie_net* net, int epochs, float lr, uint64_t seed, double* last_loss, void* stream);
/* Attach net (NULL detaches) to h for VSIE_SCHUR_LEARNED; net must outlive its use. */
int vsie_net_attach(struct vsie_handle* h, struct vsie_net* net);
/* Network passes on explicit device tensors (float32, [D][H][W][C], D, H, W multiples of 8):
 * forward of x (C = 8) into y (C = 6); loss and all parameter gradients for x and target t
 * (C = 6) with the gradients copied to grads_host (nparam floats, may be NULL); one Adam step with
 * the gradients held. Errors: E_ARG, E_NOMEM, E_HIP. */
int vsie_net_forward(struct vsie_net* net, int D, int H, int W, const float* x_dev, float* y_dev, void* stream);
int vsie_net_gradients(struct vsie_net* net, int D, int H, int W, const float* x_dev, const float* t_dev,
                       double* loss, float* grads_host, void* stream);
int vsie_net_adam(struct vsie_net* net, float lr, void* stream);
/* One layer on explicit device buffers, in the kernels' storage layout ([D][H][W][C] float32, C
 * padded to a multiple of 16 with zeros; D, H, W the layer's own grid). mode 0: forward with
 * bias and ReLU, in0 the (first) input and, for the decoder layers d3, d2, d1, in0 at half
 * resolution (upsampled in place) and in1 the skip input; out has the padded Cout channels.
 * mode 1: gradient with respect to the layer input from the output gradient in0 (masked by
 * mask > 0, mask = the layer output, for ReLU layers); out has the padded Cin channels.
 * Errors: E_ARG. */
int vsie_net_layer(struct vsie_net* net, int layer, int mode, int D, int H, int W, const float* in0,
                   const float* in1, const float* mask, float* out, void* stream);
/* Weight and bias gradients of one layer from its input(s) and output gradient g (masked by
 * mask > 0 for ReLU layers), copied to host: gw [Cout][27][Cin], gb [Cout]. Blocks. */
int vsie_net_layer_wgrad(struct vsie_net* net, int layer, int D, int H, int W, const float* in0, const float* in1,
                         const float* g, const float* mask, float* gw_host, float* gb_host, void* stream);

/* Release the handle and every device allocation it owns (operator data of eq. (15), solver and
 * elimination work space). NULL is ignored. Not thread-safe against calls on the same handle. */
void vsie_destroy(struct vsie_handle* h);
/* Message of the last failed call on this thread (empty if none); valid until the next call. */
const char* vsie_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* VSIE_H */
