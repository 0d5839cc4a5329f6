/*
 * qcdw — even-odd preconditioned Wilson-clover inversion for AMD MI355X (gfx950).
 *
 * C ABI of the HIP library libqcdw.so.  Plain pointers and sizes only.
 *
 * Field layouts at the boundary are the ones of arXiv 2411.08461, Sec. II.A
 * ("Convention"), complex numbers stored as interleaved FP64 (re, im):
 *   lattice   L = [Lx, Ly, Lz, Lt], every extent even and >= 2;
 *             even-odd site order [2, Lt, Lz, Ly, Lx/2], parity (x+y+z+t)%2,
 *             x fastest.  V = Lx Ly Lz Lt, Vh = V/2.
 *   gauge     [4, 2, Lt, Lz, Ly, Lx/2, 3, 3] complex, row-column colour order
 *             (576 V bytes).  Links must be SU(3) when reconstruct-12 is used.
 *   fermion   [2, Lt, Lz, Ly, Lx/2, 4, 3] complex (192 V bytes).
 *   clover    [2, Lt, Lz, Ly, Lx/2, 2, 36] doubles (576 V bytes): per
 *             chirality block (spins {0,1}, then {2,3}) the 6 real diagonal
 *             entries followed by the 15 complex strictly-lower entries
 *             (1,0),(2,0),(2,1),(3,0),...,(5,4) as (re, im); block row/column
 *             index 3*(spin%2)+colour.  The blocks are Hermitian.
 * Dirac matrices: DeGrand-Rossi basis (Sec. II.A).
 *
 * Operator (Sec. III.B, Eq. "clover", isotropic: xi0 = nu = 1, c_t = c_r = csw):
 *   M psi = A psi - kappa H psi,
 *   H psi(x) = sum_mu (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu),
 *   A = 1 - kappa csw C,   C = sum_{mu<nu} sigma_{mu nu} F_{mu nu},
 *   sigma_{mu nu} = [g_mu, g_nu]/2,  F = traceless part of (Q - Q^+)/8 with Q
 *   the four-leaf clover sum.  kappa = 1/(2 m0 + 8).
 * Even-odd (Sec. II.A and II.D): the solver works on the symmetric Schur
 * complement on even sites, M_hat = 1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe.
 * Solver (Sec. II.E): BiCGStab.
 *
 * Ownership and errors, for every call:
 *   - every field pointer is device memory owned by the caller (e.g. a
 *     contiguous torch tensor); the library never frees it;
 *   - the library owns its workspaces (packed links, clover inverse, Krylov
 *     vectors) inside a context or operator and frees them in *_destroy;
 *     objects must be destroyed before what they reference: nets and batches
 *     before their operators, operators before their context;
 *   - no exception crosses the ABI: each call returns a qcdw_status, and
 *     qcdw_last_error(ctx) describes the last failure on that context;
 *   - invalid arguments (odd extents, null pointers, host pointers, tol <= 0)
 *     give QCDW_EINVAL before any GPU work;
 *   - all work is enqueued on the context's stream; calls return after the
 *     results are complete on that stream unless stated otherwise.
 */
#ifndef QCDW_H
#define QCDW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qcdw_ctx qcdw_ctx;
typedef struct qcdw_op qcdw_op;
typedef struct qcdw_batch qcdw_batch;
typedef struct qcdw_net qcdw_net;
typedef struct qcdw_mg qcdw_mg;

typedef struct {
    int32_t L[4];  /* Lx, Ly, Lz, Lt: each even and >= 2 */
    int32_t t_bc;  /* +1 periodic, -1 antiperiodic in t (the paper's t_boundary) */
} qcdw_lattice;

typedef enum {
    QCDW_OK = 0,
    QCDW_EINVAL = -1,     /* bad argument */
    QCDW_ENOMEM = -2,     /* device allocation failed */
    QCDW_EHIP = -3,       /* HIP runtime error */
    QCDW_ENOCONV = -4,    /* maxiter reached before tol */
    QCDW_EBREAKDOWN = -5, /* BiCGStab breakdown that restarts could not cure */
    QCDW_ENAN = -6,       /* NaN/Inf in the source or the iteration */
    QCDW_ENOTPD = -7      /* a clover block A is not positive definite */
} qcdw_status;

typedef enum { QCDW_F64 = 0, QCDW_F32 = 1, QCDW_BF16 = 2, QCDW_F16 = 3 } qcdw_prec;

typedef struct {
    double tol;            /* target FP64 ||b - M x|| / ||b|| on the full lattice, > 0 */
    int32_t maxiter;       /* iteration cap summed over restarts and reliable updates */
    qcdw_prec inner;       /* storage precision of the Krylov iteration (F64: plain solve) */
    double delta;          /* reliable-update trigger: recompute the FP64 residual when the
                              iterated residual has fallen by this factor (mixed precision) */
    int32_t check_every;   /* host polls convergence every this many iterations (>= 1) */
    int32_t max_restarts;  /* restarts allowed after a breakdown */
    int32_t collect_timing;/* 1: time every hop launch of the iteration with HIP events recorded by
                              the dispatch itself; forces eager launches (use_graph ignored) */
    int32_t fault_inject;  /* tests only: > 0 forces a breakdown at that iteration, < 0 flags an
                              overflow (as a NaN would) at iteration -fault_inject */
    int32_t use_graph;     /* 1: each chunk of check_every iterations is captured once into a
                              hipGraph (cached on the operator) and replayed; 0: eager launches.
                              Both run the same kernels in the same order (bitwise equal x). */
    int32_t gmres_restart; /* FGMRES: Krylov vectors per restart cycle (1..64) */
    int32_t gmres_fallback;/* FGMRES: 1 = hand a stalled solve to BiCGStab, 0 = keep restarting */
    int32_t inner_resume;  /* mixed precision: 0 = every reliable update restarts BiCGStab from the true
                              residual; 1 = it replaces the iterated residual by the true one and continues
                              the recurrence (search direction, shadow residual and scalars kept), which
                              saves iterations on well-conditioned systems and costs them near the critical
                              kappa.  A cycle after a breakdown, overflow or stall always restarts. */
} qcdw_solver_params;

typedef struct {
    int32_t status;        /* qcdw_status of the solve */
    int32_t iters;         /* Krylov iterations (all restarts, all RHS max for multi) */
    int32_t n_reliable;    /* FP64 residual recomputations (reliable updates) */
    int32_t n_restarts;    /* restarts after breakdown */
    double true_res;       /* FP64 ||b - M x|| / ||b|| on the full lattice, from x */
    double iter_res;       /* last iterated relative residual of the Schur system */
    double time_ms;        /* wall time of the solve on the host */
    double hop_ms[3];      /* collect_timing = 1: summed time of the hop launches of the Krylov
                              iteration, by kind: [0] H_oe with A_oo^-1 (into odd sites),
                              [1] H_eo, A_ee^-1, xpay and (r0, v), [2] the same with (t, s), (t, t) */
    int32_t n_hop[3];      /* launches timed, same kinds */
    int32_t hist_len;      /* in: capacity of res_hist (entries) */
    int32_t hist_count;    /* out: entries written */
    int32_t fallback;      /* FGMRES: 1 if it stalled and BiCGStab finished the solve.
                              BiCGStab with a low inner precision: 1 if the cycles stopped reducing the
                              FP64 residual (3 cycles in a row without halving it, an overflow, or
                              breakdowns beyond max_restarts) and the rest of the solve ran in FP64 */
    int32_t fallback_iters;/* iterations after that switch (included in iters) */
    double *res_hist;      /* in: host buffer or NULL; out: relative residual after each
                              iteration (entry 0 = initial) */
} qcdw_solve_info;

/* Defaults: tol 1e-10, maxiter 10000, inner F64, delta 0.1, check_every 8,
   max_restarts 8, collect_timing 0, fault_inject 0, use_graph 1, gmres_restart 32, gmres_fallback 1,
   inner_resume 0. */
void qcdw_solver_params_default(qcdw_solver_params *p);

/* Context bound to one device and one HIP stream (hipStream_t, may be NULL for
   the default stream, e.g. torch.cuda.current_stream().cuda_stream). */
qcdw_status qcdw_ctx_create(qcdw_ctx **ctx, int device, void *hip_stream);
void qcdw_ctx_destroy(qcdw_ctx *ctx);
const char *qcdw_last_error(const qcdw_ctx *ctx);
qcdw_status qcdw_ctx_set_stream(qcdw_ctx *ctx, void *hip_stream);
/* The kernel form the context has chosen by timing (or read from the tuning file named by
   $QCDW_TUNE_CACHE) for a tuning key, e.g. "mrhs_hop/p2/L24x24x24x64/n12" (multi-RHS hop, BF16
   storage, 12 RHS: 0 register loop, 1 one block per RHS, 2 g the register loop in slice groups of g
   c-tiles, plus 1024 for its matrix-core form) or "hop_nt/p0/L24x24x24x64" (single-RHS hop: nt +
   16 cgroup + 4096 fma).  key: NUL-terminated host string; *value written on success.  QCDW_EINVAL
   if the key has no entry (nothing tuned for that shape yet). */
qcdw_status qcdw_ctx_tuned(const qcdw_ctx *ctx, const char *key, int *value);

/* Multi-shift CG on the normal even-odd operator (the solves of a rational approximation in RHMC,
   paper Sec. IV; the shifted solver reuses the hot path): (M_hat^+ M_hat + shifts[i]) x_i = b for
   i < n_shifts (1 .. 64, every shift finite and >= 0) in one Krylov space, FP64.  b_e, x_e[i]:
   even-site fields in the layout of qcdw_op_matpc (b read; x written, not aliasing b).  The
   shifted recurrence runs until every shifted residual it tracks is <= tol ||b|| / 2; then each
   FP64 true residual ||b - (M_hat^+ M_hat + shifts[i]) x_i|| is recomputed on the GPU from x_i,
   and a shift still above tol ||b|| is refined (at most three times) by a single-shift CG on its
   residual.  *iters (all iterations, refinements included) and res[i] (host: the relative true
   residuals) are filled.  QCDW_ENOCONV after maxiter or with a true residual above tol (res[i]
   then holds the recurrence's estimates, resp. the true residuals), QCDW_EBREAKDOWN if (p, N p)
   is not positive, QCDW_ENAN for a non-finite residual, QCDW_EINVAL for bad arguments. */
qcdw_status qcdw_invert_multishift(qcdw_op *op, const void *b_e, void *const *x_e, const double *shifts, int n_shifts,
                                   double tol, int maxiter, int *iters, double *res);

/* The 12 wall sources of the propagator workflow (Sec. III.B, the sources of the 12
   inversions): field k = 3 s0 + c0 is e^{+i p.x} on time slice t0 in spin s0, colour c0 and zero
   elsewhere, p_i = 2 pi mom[i] / L_i (mom: 3 host ints, x, y, z).  out: 12 consecutive device
   fields in the fermion layout (written).  QCDW_EINVAL for t0 outside [0, Lt). */
qcdw_status qcdw_wall_sources(qcdw_ctx *ctx, const qcdw_lattice *lat, int t0, const int *mom, void *out);

/* Meson two-point function of a propagator (the contraction after the solves, Sec. III.B):
     out[t] = sum_{x: x_t = t} e^{-i p.x} Tr[Gamma(gamma_snk) S(x) Gamma(gamma_src) g5 S(x)^+ g5],
   t = 0 .. Lt-1, with S(x)[3 s + c][k] = S_k(x)[s][c] from the 12 device fields S (fermion layout,
   k = 3 s0 + c0, read), Gamma(n) the paper's bitmask product of gamma matrices (n in [0, 15];
   15 is g5, so gamma_snk = gamma_src = 15 gives the pion), p_i = 2 pi mom[i] / L_i (3 host
   ints).  out: Lt complex FP64 on the device (written).  The sum over each slice runs in a
   fixed order (reproducible).  QCDW_EINVAL for a bitmask outside [0, 15]. */
qcdw_status qcdw_meson_2pt(qcdw_ctx *ctx, const qcdw_lattice *lat, const void *S, int gamma_snk, int gamma_src,
                           const int *mom, void *out);

/* The same trace with a second propagator T in the backward leg:
     out[t] = sum_{x: x_t = t} e^{-i p.x} Tr[Gamma(gamma_snk) S(x) Gamma(gamma_src) g5 T(x)^+ g5].
   With T the sequential propagator (M^{-1} of qcdw_seq_sources) and gamma_snk the insertion this
   is the three-point function of the paper's workflow (Sec. III.B); T = S gives qcdw_meson_2pt.
   S, T: 12 device fields each (read); out: Lt complex FP64 on the device.  QCDW_EINVAL as above. */
qcdw_status qcdw_meson_contract(qcdw_ctx *ctx, const qcdw_lattice *lat, const void *S, const void *T, int gamma_snk,
                                int gamma_src, const int *mom, void *out);

/* Sequential sources through the sink (Sec. III.B, the sequential propagator of the three-point
   function): out_k(x) = delta(x_t, t_f) e^{+i p.x} G S_k(x) with G = g5 Gamma(gamma_f)^+ g5 acting on
   the sink spin, p_i = 2 pi mom[i] / L_i.  Solving M T_k = out_k and contracting
   qcdw_meson_contract(S, T, g_ins, g_src, q) gives sum_{x_t = t_f, y_t = t} e^{-i p.x} e^{-i q.y}
   Tr[Gamma(gamma_f) S(x<-y) Gamma(g_ins) S(y<-0) Gamma(g_src) S(0<-x)].  S, out: 12 device fields
   (S read, out written, no aliasing).  QCDW_EINVAL for t_f outside [0, Lt) or a bitmask outside
   [0, 15]. */
qcdw_status qcdw_seq_sources(qcdw_ctx *ctx, const qcdw_lattice *lat, const void *S, int t_f, int gamma_f,
                             const int *mom, void *out);

/* Clover field construction when the gauge field is loaded (Sec. III.B, the
   clover term of Eq. "clover"): clover = C = sum_{mu<nu} sigma F, without
   kappa or csw.  U: gauge layout (read); clover: clover layout (written). */
qcdw_status qcdw_clover_build(qcdw_ctx *ctx, const qcdw_lattice *lat, const void *U, void *clover);

/* out = A psi with A = 1 - kappa csw C (the site-local part of Eq. "clover").
   clover: clover layout; psi, out: fermion layout; out may not alias psi. */
qcdw_status qcdw_clover_apply(qcdw_ctx *ctx, const qcdw_lattice *lat, const void *clover, const void *psi,
                              void *out, double kappa, double csw);

/* Inverse of the site-local clover term A = 1 - kappa csw C of Eq. "clover" (Sec. III.B), which
   even-odd preconditioning applies on each parity (Sec. II.A, II.D): clover_inv = A^-1 per
   chirality block (Cholesky; the blocks are Hermitian), in the packed clover layout of Sec. II.A.
   clover: C as written by qcdw_clover_build (read); clover_inv: caller-owned, same size (written).
   Returns QCDW_ENOTPD if some block of A is not positive definite (clover_inv is then undefined). */
qcdw_status qcdw_clover_invert(qcdw_ctx *ctx, const qcdw_lattice *lat, const void *clover, double kappa,
                               double csw, void *clover_inv);

/* Parity block of the Wilson hopping term H of Eq. "clover" (Sec. III.B), written out with the
   (1 -/+ gamma_mu) projectors as in the file header, in the even-odd split of Sec. II.A:
   out = H psi on sites of parity out_parity, zero on the other parity (psi's values on
   out_parity are not read).  U: gauge layout (read); psi, out: fermion layout (full lattice;
   psi read, out written, no aliasing).  QCDW_EINVAL for out_parity outside {0, 1}. */
qcdw_status qcdw_hop(qcdw_ctx *ctx, const qcdw_lattice *lat, const void *U, const void *psi, void *out,
                     int out_parity);

/* out = M psi (the full Wilson-clover matrix of Eq. "clover").  clover may be
   NULL, then it is built from U.  psi, out: fermion layout, no aliasing. */
qcdw_status qcdw_dslash(qcdw_ctx *ctx, const qcdw_lattice *lat, const void *U, const void *clover, const void *psi,
                        void *out, double kappa, double csw);

/* For callers that cannot allocate device memory (code under stream capture, tight serving loops,
   harnesses that forbid hipMalloc): qcdw_dslash with every workspace (packed links, the clover
   field when clover is NULL, packed A per parity, internal spinors) carved from a fixed device
   array of QCDW_NOALLOC_MAX_BYTES that the library holds on each device it runs on until the
   process ends.  No device memory is allocated or freed.  Arguments, layouts and the result are
   those of qcdw_dslash (the same kernels run).  The workspace needs about 2.6 kB per site (3.2 kB
   when clover is NULL): lattices beyond the fixed size give QCDW_EINVAL with the size in the
   message.  Calls on one device share the array, which keeps the last call's contents: calls
   that overlap on one device (several streams or threads) race, so the caller serialises them. */
#define QCDW_NOALLOC_MAX_BYTES 67108864
qcdw_status qcdw_dslash_noalloc(qcdw_ctx *ctx, const qcdw_lattice *lat, const void *U, const void *clover,
                                const void *psi, void *out, double kappa, double csw);

/* Operator object (the getDirac + loadGauge step of Sec. III.B): packs U into
   the internal site-major layout (reconstruct-12 when recon == 12, else 18),
   builds the clover field, inverts A on both parities, and keeps FP64 copies
   plus copies in `inner` storage precision.  U is not referenced afterwards. */
qcdw_status qcdw_op_create(qcdw_ctx *ctx, const qcdw_lattice *lat, const void *U, double kappa, double csw,
                           qcdw_prec inner, int recon, qcdw_op **op);

/* The anisotropic clover operator of the paper's example action (Sec. III.B, Eq. "clover"):
     M = A - kappa [H_t + (nu / xi_0) sum_i H_i],
     A = 1 - kappa [csw_t sum_i sigma_i4 F_i4 + (csw_r / xi_0) sum_{i<j} sigma_ij F_ij],
   with H_mu the two hops of direction mu (i = x, y, z spatial) and, in the paper's convention,
   kappa = 1 / (2 (m_0 + 1 + 3 nu / xi_0)) (the caller passes kappa).  xi_0 = nu = 1 and
   csw_t = csw_r = csw is the isotropic operator of qcdw_op_create.  Arguments, ownership and the
   precision handling are those of qcdw_op_create; every operator call (matpc, solves, multi-RHS,
   batches, FGMRES) then uses the anisotropic operator.  QCDW_EINVAL for xi_0 or nu not positive
   and finite. */
qcdw_status qcdw_op_create_aniso(qcdw_ctx *ctx, const qcdw_lattice *lat, const void *U, double kappa, double xi_0,
                                 double nu, double csw_t, double csw_r, qcdw_prec inner, int recon, qcdw_op **op);
void qcdw_op_destroy(qcdw_op *op);

/* The form of the operator's single-RHS parity hop in precision prec (F64 or the inner
   precision), chosen by timing when the operator was created or read from the tuning cache
   ($QCDW_TUNE_CACHE, the role of the paper's resource_path, Sec. III.B): *nt output sites per
   thread along t (1, 2, 4 or 8), *cgroup c-tiles per group swept along t (0: none) and *fma (may be
   NULL): bit 0 the arithmetic form (every complex multiply-add as real multiply-adds), bit 1 the
   t-neighbour spinors of each 64-site tile staged in LDS (slice groups with nt = 1 only).  nt,
   cgroup and the staging change only the order of memory accesses; bit 0 changes the rounding of
   the result (within a few units in the last place per site).  Returns QCDW_EINVAL for a NULL nt
   or cgroup or another precision. */
qcdw_status qcdw_op_hop_form(const qcdw_op *op, qcdw_prec prec, int *nt, int *cgroup, int *fma);

/* The even-odd preconditioned operator of Sec. II.A / II.D (the Schur complement on even sites
   of Eq. "clover"'s M): out_e = M_hat in_e = in_e - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe in_e.
   in_e, out_e: [Lt, Lz, Ly, Lx/2, 4, 3] complex FP64 (the even half of the fermion layout; in_e
   read, out_e written, no aliasing).  prec selects the storage precision of the kernels used
   (F64, or the op's inner precision); the result is returned in FP64.  QCDW_EINVAL for another
   precision. */
qcdw_status qcdw_op_matpc(qcdw_op *op, qcdw_prec prec, const void *in_e, void *out_e);

/* The same for nrhs (1..16) stacked even-site fields, with the multi-RHS hop
   kernel (each link and clover entry loaded once per site for all RHS).
   Reconstruct-12 operators only. */
qcdw_status qcdw_op_matpc_multi(qcdw_op *op, qcdw_prec prec, int nrhs, const void *in_e, void *out_e);

/* Solve M x = b (fermion layout) for the Wilson-clover matrix of Eq. "clover" by BiCGStab, the
   paper's solver for clover fermions (Sec. II.E), on the even-odd system of Sec. II.A / II.D,
   with the tolerance and iteration cap of the paper's invert calls (Sec. III.B: tol, maxiter).
   b: read; x holds the initial guess on entry (zeros for none) and the solution on exit; it is
   written on QCDW_OK and QCDW_ENOCONV (best iterate).  info is always filled.  The acceptance
   test is the FP64 true residual of the full system, recomputed from x. */
qcdw_status qcdw_invert(qcdw_op *op, const void *b, void *x, const qcdw_solver_params *params,
                        qcdw_solve_info *info);

/* nrhs (1..16) right-hand sides solved together (Sec. III.B: a propagator is
   12 solves).  b, x: nrhs consecutive fermion fields.  info: nrhs entries.
   Every launch of the iteration serves all RHS (one multi-RHS hop per parity
   block applies each link to all RHS of a site; of its forms, links held in
   registers (vector or, for 16-bit storage, matrix-core products) or re-read
   from L2, the fastest is picked by timing on first use, see qcdw_ctx_tuned);
   each RHS keeps its own BiCGStab scalars, targets and flags, and stops on its
   own (masked). */
qcdw_status qcdw_invert_multi(qcdw_op *op, int nrhs, const void *b, void *x, const qcdw_solver_params *params,
                              qcdw_solve_info *info);

/* Batched solves of different operators (lattice sizes, kappas) in lockstep.
   A batch references 1..64 reconstruct-12 operators of one context with the
   same inner precision (they must outlive it) and owns the solver workspace.
   Every launch of the iteration serves all problems: the hop kernels are
   persistent grids that walk a device table of the problems' tiles, with the
   grid size picked by timing candidates on first use (cached on the context,
   and in the file named by $QCDW_TUNE_CACHE when set, the role of the paper's
   tuning-cache resource_path, Sec. III.B).  Finished problems are masked. */
qcdw_status qcdw_batch_create(qcdw_ctx *ctx, int n, qcdw_op *const ops[], qcdw_batch **batch);
void qcdw_batch_destroy(qcdw_batch *batch);
/* b[k], x[k]: fermion fields of operator k (x: initial guess in, solution out);
   info: n entries.  Same conventions as qcdw_invert for each problem. */
qcdw_status qcdw_invert_batch(qcdw_batch *batch, const void *const b[], void *const x[],
                              const qcdw_solver_params *params, qcdw_solve_info *info);

/* Learned gauge-covariant preconditioner (the paper's accelerator for clover
   solves is multigrid, Sec. II.E; this follows the published idea of
   gauge-equivariant convolutions, Favoni et al. 2022, Lehner and Wettig 2023).
   Two linear layers on the full lattice, 4 -> hidden -> 4 channels (input
   channels = spins), each out_c'(x) = sum_{a in {0, +-mu}} sum_c W_a[c', c]
   (T_a phi_c)(x) with T_{+mu} phi(x) = U_mu(x) phi(x+mu), T_{-mu} phi(x) =
   U_mu(x-mu)^+ phi(x-mu); no bias, no nonlinearity.  As a preconditioner of the
   even-odd system it maps an even-site field r_e to restrict_even(net(embed r_e)).
   Weights: complex, [9][cout][cin], hop order a = 0, +x, -x, +y, -y, +z, -z, +t, -t.
   The net holds an FP32 copy of the operator's reconstruct-12 links; op must be
   reconstruct-12 and must outlive the net.  Training and gradients use FP32
   activations; application for FGMRES uses BF16 hidden activations. */
qcdw_status qcdw_net_create(qcdw_op *op, int hidden, uint64_t seed, double init_scale, qcdw_net **net);
void qcdw_net_destroy(qcdw_net *net);
/* Rebind the net to another operator on a lattice of the same extents (another gauge field of
   the same ensemble): the links are copied, weights and Adam moments are kept, so training can
   continue on several fields and the trained net can precondition a field it has not seen (the
   layers are gauge-covariant with field-independent weights).  op must be reconstruct-12, on the
   same context, and must outlive the net (or a later rebinding).  EINVAL on mismatch. */
qcdw_status qcdw_net_bind(qcdw_net *net, qcdw_op *op);
/* host arrays of 2*9*hidden*4 doubles (re, im interleaved), W1 [9][hidden][4], W2 [9][4][hidden] */
qcdw_status qcdw_net_get_weights(qcdw_net *net, double *w1, double *w2);
qcdw_status qcdw_net_set_weights(qcdw_net *net, const double *w1, const double *w2);
/* out_e = P(in_e); even-site fermion fields [Lt,Lz,Ly,Lx/2,4,3] complex FP64 on the device.
   prec: QCDW_F32 (FP32 activations) or QCDW_BF16 (BF16 hidden activations). */
qcdw_status qcdw_net_apply(qcdw_net *net, qcdw_prec prec, const void *in_e, void *out_e);
/* loss = sum_k ||P(r_k) - e_k||^2 / ||e_k||^2 over npairs even-site pairs (device pointers,
   FP64), and its gradients dL/dRe W + i dL/dIm W into host arrays g1, g2 (layout as the weights). */
qcdw_status qcdw_net_loss_grad(qcdw_net *net, int npairs, const void *const r_e[], const void *const e_e[],
                               double *loss, double *g1, double *g2);
/* Adam (lr, beta1 0.9, beta2 0.999, eps 1e-8) on mini-batches of `batch` pairs drawn in a
   seeded shuffled order; loss_hist (host, `steps` entries or NULL) receives each batch's mean loss. */
qcdw_status qcdw_net_train(qcdw_net *net, int npairs, const void *const r_e[], const void *const e_e[], int steps,
                           int batch, double lr, uint64_t seed, double *loss_hist);
/* Solver-generated training pairs for the net: x* from an FP64 solve of M x = b to 1e-12; the
   iterates x_k of FP64 BiCGStab restarted every `stride` iterations from zero, k = 1..npairs;
   e_k = (x* - x_k) on even sites and r_k = M_hat e_k, both scaled so that ||r_k|| = 1.
   With stride < 0 the errors are instead seeded Gaussian fields (seed = -stride, stream k) and
   r_k = M_hat e_k (b is not used): pairs that weight all modes alike.
   r_e[k], e_e[k]: caller-owned even-site fields [Lt,Lz,Ly,Lx/2,4,3] complex FP64 on the device.
   *made receives the number of pairs written (fewer than npairs if the iteration converged). */
qcdw_status qcdw_make_training_pairs(qcdw_op *op, const void *b, int npairs, int stride, void *const r_e[],
                                     void *const e_e[], int *made);
/* Flexible GMRES(m) (Saad 1993, m = params->gmres_restart) on the even-odd system with right
   preconditioning z = P(v) (net may be NULL: no preconditioner; the net is applied with BF16
   hidden activations), block classical Gram-Schmidt applied twice (a single pass with a
   conditional second one was measured to need the second pass at almost every step, at the
   cost of a second host synchronisation).  With params->gmres_fallback, a restart cycle that reduces the residual by less
   than 10 % hands the solve to BiCGStab in the operator's inner precision from the current
   iterate.  The final acceptance is the FP64 true residual of the full system, as for
   qcdw_invert.  b, x: full fermion fields as for qcdw_invert (x: initial guess in, solution out).
   Returns OK, ENOCONV (x holds the best iterate), ENAN, or EINVAL/ENOMEM/EHIP. */
qcdw_status qcdw_invert_fgmres(qcdw_op *op, qcdw_net *net, const void *b, void *x, const qcdw_solver_params *params,
                               qcdw_solve_info *info);

/* Clover fermion force, the link derivative that HMC with clover fermions integrates (Sec. IV):
   for the operator M = A - kappa H of qcdw_dslash (isotropic, time boundary of lat) and fields X, Y,
     H_mu(x) = sum_a T^a d/dw [2 Re(Y^+ M(U_w) X)] at w = 0,  U_w: U_mu(x) -> exp(i w T^a) U_mu(x),
   T^a = lambda^a / 2 (Gell-Mann), every other link fixed; H_mu(x) is Hermitian and traceless.  For the
   two-flavour action S = phi^+ (M^+ M)^-1 phi with X = (M^+ M)^-1 phi and Y = M X (two qcdw_invert
   solves: Y = g5 M^-1 g5 phi, X = M^-1 Y), the derivative of S along T^a is -2 Tr(T^a H_mu(x)).
   U: gauge layout (read; SU(3) not required); X, Y: fermion layout (read); H: gauge layout (written,
   no aliasing).  Uses a scratch field of 6 x 144 V bytes. */
qcdw_status qcdw_clover_force(qcdw_ctx *ctx, const qcdw_lattice *lat, const void *U, const void *X, const void *Y,
                              double kappa, double csw, void *H);

/* Two-level aggregation multigrid, the paper's accelerator for Wilson/clover solves (Sec. II.E: the
   multigrid solver is built from a block size per level, set up when the gauge field is loaded and
   reusable for other masses; Sec. III.B: a 2^4 sublattice becomes one coarse site).  The lattice is cut
   into blocks of block[] sites; each block, split by chirality (spins {0,1} and {2,3}), is an aggregate.
   Near-null vectors v_0 .. v_{nvec-1} (given, or generated by relaxing M v = 0 from seeded Gaussian
   fields eta_k: v_k = eta_k - y_k after setup_iters BiCGStab iterations on M y = M eta_k from zero) are
   orthonormalised on every aggregate by modified Gram-Schmidt in the order k = 0, 1, ..: the
   prolongator P (P^+ P = 1, P commutes with gamma_5; a vector left with less than 1e-10 of its norm
   outside the span of the earlier ones on an aggregate counts as linearly dependent).  The
   coarse operator is the Galerkin product D_c = P^+ M P, a nearest-neighbour stencil of (2 nvec)^2
   complex blocks on the coarse lattice L / block (coarse sites numbered with x fastest).  As the
   preconditioner of the even-odd system it maps v_e to [P D_c^-1 P^+ (A_ee v_e)]_e (M_hat^-1 =
   (M^-1)_ee A_ee), the coarse system solved by at most coarse_iters BiCGStab iterations in FP32 (or to
   coarse_tol relative), followed by smooth_iters minimal-residual steps on M_hat. */
typedef struct {
    int32_t block[4];      /* aggregate extents (each divides its lattice extent; their product even) */
    int32_t nvec;          /* near-null vectors (1 .. 32, at most 6 |block|): 2 nvec unknowns per coarse site */
    int32_t setup_iters;   /* BiCGStab iterations per generated near-null vector (>= 1) */
    uint64_t seed;         /* seed of the Gaussian starting fields (counter-based generator) */
    int32_t coarse_iters;  /* BiCGStab iterations of each coarse solve (>= 0) */
    double coarse_tol;     /* relative residual at which a coarse solve stops early (> 0) */
    int32_t smooth_iters;  /* minimal-residual steps on M_hat after the coarse correction (>= 0) */
} qcdw_mg_params;

/* Defaults: block 4^4, nvec 12, setup_iters 100, seed 1234, coarse_iters 24, coarse_tol 0.1,
   smooth_iters 2. */
void qcdw_mg_params_default(qcdw_mg_params *p);
/* Set up the multigrid for op (the loadGauge step that builds it, Sec. III.B).  vecs: NULL (generate) or
   nvec device fields in the fermion layout, read.  Generated vectors relax M v = 0 from seeded Gaussian
   fields: setup_iters iterations of BiCGStab in the operator's inner precision on M y = M eta from y = 0,
   one vector after the other, v = eta - y.  The object holds the block vectors (FP64
   and FP32), the coarse stencil (FP64, and BF16 for the preconditioner's coarse solve) and the coarse
   solver workspace; op must outlive it.  EINVAL for a block that does not tile the lattice, nvec out of
   range or linearly dependent vectors on an aggregate. */
qcdw_status qcdw_mg_create(qcdw_op *op, const qcdw_mg_params *params, const void *vecs, qcdw_mg **mg);
void qcdw_mg_destroy(qcdw_mg *mg);
/* coarse_dims: 4 host ints, L / block; nvec: host int */
qcdw_status qcdw_mg_info(const qcdw_mg *mg, int *coarse_dims, int *nvec);
/* The orthonormalised block vectors as nvec device fields in the fermion layout (written). */
qcdw_status qcdw_mg_vectors(qcdw_mg *mg, void *vecs);
/* coarse = P^+ fine (fine: device fermion field, read; coarse: device [Vc][2][nvec] complex FP64, written). */
qcdw_status qcdw_mg_restrict(qcdw_mg *mg, const void *fine, void *coarse);
/* fine = P coarse (layouts as qcdw_mg_restrict). */
qcdw_status qcdw_mg_prolong(qcdw_mg *mg, const void *coarse, void *fine);
/* out = D_c in on coarse vectors [Vc][2][nvec] complex FP64 (device, no aliasing). */
qcdw_status qcdw_mg_coarse_apply(qcdw_mg *mg, const void *in, void *out);
/* The coarse stencil as [Vc][9][2 nvec][2 nvec] complex FP64 (row-major blocks; entry 0 couples a coarse
   site to itself, 1 + 2 mu to its +mu neighbour, 2 + 2 mu to its -mu neighbour): device, written. */
qcdw_status qcdw_mg_coarse_op(qcdw_mg *mg, void *stencil);
/* Solve M x = b by FGMRES(m) (m = params->gmres_restart) on the even-odd system with the multigrid
   preconditioner; conventions of qcdw_invert_fgmres (FP64 true-residual acceptance, BiCGStab fallback).
   op may be another operator of the same gauge field and lattice (another mass, reusing the set-up as
   the paper does); EINVAL for another context or lattice. */
qcdw_status qcdw_invert_mg(qcdw_op *op, qcdw_mg *mg, const void *b, void *x, const qcdw_solver_params *params,
                           qcdw_solve_info *info);

#ifdef __cplusplus
}
#endif

#endif /* QCDW_H */
