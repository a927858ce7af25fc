/*
 * kubo.h -- C ABI of the MI355X (gfx950) Kubo-formula library.
 *
 * The library evaluates the intrinsic anomalous Hall conductivity sigma_xy of
 * tight-binding models on a uniform Brillouin-zone grid, following the paper's
 * Eqs. (2)-(3) and the four per-k steps of its baseline listing: build the
 * Bloch Hamiltonian H(k) and the velocities dH/dk_a from the hoppings t(R),
 * diagonalise H(k), rotate the velocities into the eigenbasis, and sum the
 * band-pair Berry curvature weighted by the occupations.  Many k-points (and
 * many models) are processed as one batch, the idea of the paper's
 * "vectorized implementation" section and its Eq. (4); the batched sum equals
 * the plain one up to summation order.
 *
 * Conventions used by every entry point
 *   - k = 2 pi (i0/N0, i1/N1, i2/N2), a Gamma-centred grid; the flat k index is
 *     f = i0 + N0 (i1 + N1 i2).  Lattice vectors R are integer triples in a
 *     cubic cell of unit length.
 *   - Ht = sum_R t(R) e^{i k.R}, H = (Ht + Ht^+)/2, and likewise for the
 *     velocities vt_a = sum_R i R_a t(R) e^{i k.R}; only the Hermitian part of
 *     the Bloch sum enters, so every entry of t is an independent parameter.
 *   - g(x) = 1/(x^2 + eta^2) regularises the band-pair denominator of Eq. (3);
 *     occupations are Fermi-Dirac at kT > 0 and a step (with f = 1/2 exactly
 *     at E = E_F) at kT = 0.
 *   - sigma_xy[j] = -(1/N_k) sum_k sum_n f(E_n; E_F[j]) Omega_n(k), with
 *     Omega_n = -2 sum_{m != n} Im(A_nm B_mn) g(E_n - E_m), A = U^+ v_x U,
 *     B = U^+ v_y U; units e^2/hbar per lattice constant.  N_k is the FULL
 *     grid even when a k-slab is requested, so disjoint slabs add up.
 *   - All floating point is IEEE binary64.  Complex arrays are interleaved
 *     (re, im) doubles.  t is [n_R][n][n] row-major per model; the models of a
 *     plan are concatenated in plan order.
 *   - Device pointers are HIP device memory owned by the caller.  "stream" is
 *     a hipStream_t (NULL = the default stream).  Calls only enqueue work; a
 *     non-OK return means nothing was enqueued.  Results are bitwise identical
 *     from run to run (fixed reduction order, no floating-point atomics).
 *   - The library never allocates device memory: the caller passes a
 *     workspace of at least the size kubo_plan reports.  A call uploads the
 *     plan's index tables into the workspace, and synchronises the stream,
 *     when that workspace does not hold them already (its first use by the
 *     plan, or another plan ran on it since); plans may therefore take turns
 *     on one workspace.  The caller must not modify a workspace between calls.
 *   - A plan is not safe to use from two threads at once.
 */
#ifndef KUBO_H
#define KUBO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kubo_plan_s* kubo_plan_t;

typedef enum {
    KUBO_OK = 0,
    KUBO_E_INVALID = 1,     /* an argument is out of its documented range */
    KUBO_E_UNSUPPORTED = 2, /* valid, but beyond what this library implements */
    KUBO_E_WORKSPACE = 3,   /* workspace NULL or smaller than kubo_plan reported */
    KUBO_E_HIP = 4,         /* a HIP runtime call failed (launch, copy, graph) */
    KUBO_E_NOCONV = 5,      /* device: an eigensolve hit its sweep cap */
    KUBO_E_NONFINITE = 6    /* device: a non-finite value reached the result */
} kubo_status;

/* One tight-binding model and the part of its k-grid to sum over. */
typedef struct {
    int32_t n_orb;        /* orbitals n (matrix size), 1 <= n <= 512; n > 128 runs the
                             large-n pipeline (forward only, see kubo_plan) */
    int32_t n_R;          /* number of lattice vectors, >= 1 */
    const int32_t* R;     /* HOST array [n_R][3]; no duplicates, closed under R -> -R.
                             Copied by kubo_plan. */
    int32_t grid[3];      /* N0, N1, N2 >= 1 */
    int64_t k_begin;      /* first flat k index of the slab, 0 <= k_begin < N_k */
    int64_t k_count;      /* k-points in the slab; -1 means "to the end of the grid" */
} kubo_model_desc;

/* Per-orbital-count launch shape; the autotuner writes these. */
typedef struct {
    int32_t n_orb;        /* the models with this n use the entry */
    int32_t threads;      /* 0 = default; 64 = one wavefront per k-point (n <= 32 only);
                             256 = one 256-thread workgroup per k-point */
    int32_t k_block;      /* k-points per work item (a piece of one kx pencil), >= 1 */
    int32_t reserved;     /* must be 0 */
} kubo_tile;

/* kubo_plan flags */
#define KUBO_F_GRAPH 0x1u        /* capture each call's launches in a hipGraph and replay it
                                    while the pointers and scalars stay the same */
#define KUBO_F_TIMING 0x2u       /* record HIP events around every launch of the per-k
                                    kernels (ignored while KUBO_F_GRAPH replays) */
#define KUBO_F_FORWARD_ONLY 0x4u /* size the workspace for kubo_ahc only; kubo_ahc_backward
                                    then returns KUBO_E_INVALID */
#define KUBO_F_TENSOR 0x8u       /* size the workspace for kubo_ahc_tensor as well (a third
                                    set of partial Bloch sums, four result components) */
#define KUBO_F_DEBUG_SWEEPCAP 0x100u /* cap the iterative eigensolver at one iteration (one
                                    sweep) and route every k-point through it, so that the
                                    device status reports KUBO_E_NOCONV (tests of that path) */

/*
 * kubo_plan -- validate the models and build the host-side plan.  No device
 * work and no device allocation happen here; it runs without a GPU.
 *   plan            out: the new plan (unchanged on error)
 *   models          host array of n_models descriptors
 *   n_models        >= 1
 *   n_fermi         Fermi levels per model, 1 <= n_fermi <= 4096
 *   flags           KUBO_F_* bits; unknown bits are KUBO_E_INVALID
 *   tiles, n_tiles  optional launch shapes (NULL/0 = built-in defaults)
 *   workspace_bytes out: device workspace the plan needs (forward and backward,
 *                   or forward only with KUBO_F_FORWARD_ONLY)
 * The k-grid is processed in chunks of kx pencils whose partial Bloch sums fit
 * a buffer of KUBO_CHUNK_MB megabytes (environment variable read here; default
 * 2048); the backward's per-k-block pencil partials and per-k adjoint
 * matrices get four times that.
 * Larger chunks mean fewer launches and a larger workspace.
 * Errors: KUBO_E_INVALID for NULL pointers, n_orb < 1, n_R < 1, grid < 1,
 * duplicate R, an R whose negative is missing, a slab outside the grid or a
 * bad tile; KUBO_E_UNSUPPORTED for n_orb > 512, for more than 16 distinct R_x,
 * and for a model with n_orb > 128 in a plan without KUBO_F_FORWARD_ONLY or with
 * KUBO_F_TENSOR.  Models with 128 < n_orb <= 512 (the paper's large-N_d regime,
 * end of its section on the vectorised implementation) run a pipeline that
 * spreads each k-point over many workgroups: Householder reduction, bisection on
 * the split tridiagonal matrix, tridiagonal eigenvectors, a compact-WY
 * back-transformation and the rotations on batched matrix-core products; their
 * per-k-point slices (about 12 n^2 complex elements each, for up to KUBO_BIG_BATCH
 * k-points at a time: environment variable read here, default 256, 1..4096) are
 * part of the workspace.
 */
kubo_status kubo_plan(kubo_plan_t* plan, const kubo_model_desc* models, int32_t n_models,
                      int32_t n_fermi, uint32_t flags, const kubo_tile* tiles, int32_t n_tiles,
                      size_t* workspace_bytes);

/*
 * kubo_ahc -- sigma_xy (paper Eqs. (2)-(3)) for every model and Fermi level.
 *   t          device, complex128: the models' t arrays concatenated in plan order
 *   e_fermi    device, double [n_models][n_fermi]
 *   eta        broadening, >= 0 (finite)
 *   kT         temperature in energy units, >= 0 (finite); 0 selects the step
 *   sigma      device, double [n_models][n_fermi], overwritten
 *   workspace  device, >= workspace_bytes of kubo_plan
 * Errors: KUBO_E_INVALID (NULL pointers, eta or kT negative or not finite),
 * KUBO_E_WORKSPACE, KUBO_E_HIP.  Eigensolver non-convergence and non-finite
 * results are reported later by kubo_plan_device_status.
 */
kubo_status kubo_ahc(kubo_plan_t plan, const double* t, const double* e_fermi, double eta,
                     double kT, double* sigma, void* workspace, size_t workspace_bytes,
                     void* stream);

/*
 * kubo_ahc_tensor -- the general response of the paper's Eq. (1) for other pairs
 * of current operators, in one pass (one eigendecomposition per k-point): the
 * anomalous Hall tensor and the spin Hall conductivity.  For the operator pair
 * (P, Q) with P' = U^+ P U, Q' = U^+ Q U:
 *   sigma_PQ[j] = -(1/N_k) sum_k sum_n f(E_n; E_F[j]) Omega^PQ_n,
 *   Omega^PQ_n  = -2 sum_{m != n} Im(P'_nm Q'_mn) g(E_n - E_m)
 * (Eq. (3) with its two current operators replaced), for the four pairs
 *   c = 0: (v_x, v_y) = sigma_xy (equal to kubo_ahc's result, bit for bit)
 *   c = 1: (v_y, v_z) = sigma_yz      c = 2: (v_z, v_x) = sigma_zx
 *   c = 3: (Js_x, v_y), the spin Hall conductivity, with the spin current
 *          Js_x = (s_z v_x + v_x s_z)/2 and s_z = diag(spin) in the orbital basis
 *          (spin in the caller's units, e.g. +1/-1 for up/down)
 * v_z = sum_R i R_z t(R) e^{ik.R} (Hermitian part), like v_x and v_y.
 *   t, e_fermi, eta, kT, workspace as for kubo_ahc
 *   spin       device, double [sum of n_orb over the models] (the models' orbitals in
 *              plan order), or NULL: then component 3 is zero and not computed
 *   sigma      device, double [n_models][4][n_fermi], overwritten
 * The plan must carry KUBO_F_TENSOR (else KUBO_E_INVALID).  Errors: as kubo_ahc.
 */
kubo_status kubo_ahc_tensor(kubo_plan_t plan, const double* t, const double* e_fermi, double eta,
                            double kT, const double* spin, double* sigma, void* workspace,
                            size_t workspace_bytes, void* stream);

/* most quadrature nodes of one kubo_ahc_gf call */
#define KUBO_GF_MAX_NODES 65536

/*
 * kubo_ahc_gf -- the Green's-function form of sigma_xy, which the paper names
 * (remark after Eq. (3)) for systems with impurities: matrix inverses in place of
 * the eigendecomposition.  With a constant scattering rate gamma,
 *   G(w)       = ((i (w + gamma) + E_F[j]) I - H(k))^{-1}
 *   sigma[j]   = (1/N_k) sum_k sum_l weight[l] Im{Tr[G v_x G G v_y] - Tr[G v_y G G v_x]} / (2 pi)
 * with G = G(omega[l]): a quadrature over w > 0 given by the caller.  With
 * gamma = 0 and a converged quadrature this is kubo_ahc's sigma_xy at eta = 0,
 * kT = 0 (the residues of the poles at w = i (E_F - E_n) give Eq. (3)).
 *   t, e_fermi, workspace as for kubo_ahc; the plan may be any plan of models
 *              with n_orb <= 32 (else KUBO_E_UNSUPPORTED)
 *   gamma      >= 0 (finite)
 *   omega      device, double [n_omega]: the nodes; omega[l] + gamma > 0 keeps
 *              every G finite (a zero would be reported as KUBO_E_NONFINITE)
 *   weight     device, double [n_omega]: the weights
 *   n_omega    1 <= n_omega <= KUBO_GF_MAX_NODES
 *   sigma      device, double [n_models][n_fermi], overwritten
 * One inverse (Gauss-Jordan elimination, no pivoting: i (w + gamma) + E_F - H has
 * the positive definite part w + gamma along i) and four matrix products per
 * k-point, Fermi level and node.  Errors: as kubo_ahc.
 */
kubo_status kubo_ahc_gf(kubo_plan_t plan, const double* t, const double* e_fermi, double gamma,
                        const double* omega, const double* weight, int32_t n_omega, double* sigma,
                        void* workspace, size_t workspace_bytes, void* stream);

/*
 * kubo_ahc_backward -- gradient of L = sum_{m,j} sigma_bar[m][j] sigma[m][j]
 * with respect to every hopping: grad_t = dL/dRe t + i dL/dIm t (the
 * convention of complex autograd), by reverse-mode differentiation through
 * the eigendecomposition.  Eigenvectors are recomputed per k-block rather
 * than stored.  Same arguments as kubo_ahc, plus
 *   sigma_bar  device, double [n_models][n_fermi]
 *   grad_t     device, complex128, laid out like t, overwritten
 * eta must be > 0 (the curvature denominator needs it).  At kT = 0 the
 * Fermi-surface term (derivative of the step) is omitted.
 * Errors: as kubo_ahc; eta == 0 is KUBO_E_INVALID.
 */
kubo_status kubo_ahc_backward(kubo_plan_t plan, const double* t, const double* e_fermi,
                              double eta, double kT, const double* sigma_bar, double* grad_t,
                              void* workspace, size_t workspace_bytes, void* stream);

/*
 * kubo_plan_device_status -- synchronise the stream and report what the
 * kernels of the last call on this workspace flagged: KUBO_E_NOCONV,
 * KUBO_E_NONFINITE (NOCONV wins if both), or KUBO_OK.  KUBO_E_HIP if the
 * synchronisation or the read fails; KUBO_E_INVALID before any call.
 */
kubo_status kubo_plan_device_status(kubo_plan_t plan, const void* workspace, void* stream);

/* Free the plan (host memory and any captured graph).  NULL is a no-op. */
void kubo_plan_destroy(kubo_plan_t plan);

/* A static, human-readable name for a status code. */
const char* kubo_status_string(kubo_status status);

/*
 * kubo_plan_kernel_time -- device time of the per-k kernels recorded under
 * KUBO_F_TIMING since the last reset.  which = 0: the forward per-k kernel
 * (Bloch sum, eigensolve, rotation, curvature and Fermi sums); which = 1: the
 * backward per-k kernel; which = 2: the per-k kernel of kubo_ahc_tensor; which
 * = 3: the per-k kernel of kubo_ahc_gf; which = 4: the Householder reduction
 * kernel of the large-n path alone (which = 0 covers its whole pipeline).  Waits
 * for the recorded events.  Outputs (each may
 * be NULL): total_ms, the number of launches, and the k-points they covered.
 * reset != 0 forgets the records afterwards.  KUBO_E_INVALID for a NULL plan
 * or a bad which; KUBO_E_HIP if an event query fails.
 */
kubo_status kubo_plan_kernel_time(kubo_plan_t plan, int32_t which, double* total_ms,
                                  int64_t* launches, int64_t* k_points, int32_t reset);

/* Work totals of a plan, for throughput reports: k-points summed over all
 * models and slabs, and the number of models.  Returns KUBO_E_INVALID on NULL. */
kubo_status kubo_plan_info(kubo_plan_t plan, int64_t* total_k_points, int32_t* n_models);

/* Size of the library's own device workspace used by kubo_ahc_noalloc. */
#define KUBO_NOALLOC_MAX_BYTES (64u << 20)

/* Device status bits that kubo_ahc_noalloc can report. */
#define KUBO_DEVICE_NOCONV 0x1u
#define KUBO_DEVICE_NONFINITE 0x2u

/*
 * kubo_ahc_noalloc -- kubo_ahc without a caller workspace, for callers that
 * cannot allocate device memory (code that must not call hipMalloc, tight
 * serving loops, harnesses that forbid allocation).  The workspace is a
 * static device array inside the library, KUBO_NOALLOC_MAX_BYTES per GPU,
 * held until the process ends; nothing is allocated or freed by the call.
 *   plan, t, e_fermi, eta, kT, sigma   as for kubo_ahc (same results, bit for bit)
 *   device_status  device uint32_t, or NULL: receives the device-side status
 *                  bits of this call (0, or KUBO_DEVICE_NOCONV and/or
 *                  KUBO_DEVICE_NONFINITE), written on the stream
 *   stream         a stream of the current device
 * Every call on one GPU shares that GPU's array, so calls that overlap in
 * time on one GPU (two streams, two threads) race and give wrong results;
 * calls on one stream are safe.  The plan's tables are uploaded (and the
 * stream synchronised) when the array last held another plan's.  Always
 * eager: KUBO_F_GRAPH and KUBO_F_TIMING are ignored here.
 * Errors: as kubo_ahc; KUBO_E_WORKSPACE when the plan's workspace_bytes
 * exceed KUBO_NOALLOC_MAX_BYTES (plan with KUBO_F_FORWARD_ONLY and, for large
 * grids, a smaller KUBO_CHUNK_MB); KUBO_E_HIP if the array's address cannot
 * be found on the current device.
 */
kubo_status kubo_ahc_noalloc(kubo_plan_t plan, const double* t, const double* e_fermi,
                             double eta, double kT, double* sigma, uint32_t* device_status,
                             void* stream);

#ifdef __cplusplus
}
#endif

#endif /* KUBO_H */
