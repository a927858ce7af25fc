/*
 * kubo_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE LIBRARY.
 *
 * A plain, slow, FP64 CPU oracle for the intrinsic anomalous Hall
 * conductivity sigma_xy of a tight-binding model, evaluated by the Kubo
 * formula on a uniform Brillouin-zone grid.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or helper with the HIP library; the two meet only in
 * the seeded input generator.
 *
 * What it follows (paper, "Numerical method"):
 *   - Eq. (1) and the text under it: an equilibrium average becomes a
 *     Brillouin-zone integral (2 pi)^-3 V \int dk Tr X(k); on a uniform grid of
 *     N_k points with a unit cubic cell this is (1/N_k) sum_k.
 *   - Eq. (2)-(3): sigma is a k-sum of a band-pair sum of
 *     Im(J_nm J_mn) / (E_m - E_n)^2 weighted by the occupation of band n.
 *   - The baseline listing's four per-k steps: build H(k) and the current
 *     operators, diagonalise H, rotate the currents into the eigenbasis,
 *     evaluate the band-pair sum and accumulate.
 * Readings where the paper is silent (current = dH/dk with e = hbar = 1,
 * sigma_xy = -sigma_yx, broadening g(x) = 1/(x^2+eta^2), Fermi-Dirac
 * occupation for kT > 0 with theta(0) = 1/2 at kT = 0, Hermitian projection
 * of the Bloch sum, Gamma-centred grid) are listed in the design notes.
 *
 * Definition computed by oracle_ahc (pair form; equal to -(1/N_k) sum_k sum_n
 * f_n Omega_n by the antisymmetry of Im(A_nm B_mn) in n <-> m):
 *   k        = 2 pi (i0/N0, i1/N1, i2/N2), flat index f = i0 + N0 (i1 + N1 i2)
 *   Ht       = sum_R t(R) e^{i k.R},  vt_a = sum_R i R_a t(R) e^{i k.R}
 *   H        = (Ht + Ht^+)/2,          v_a  = (vt_a + vt_a^+)/2
 *   H        = U diag(E) U^+           (own cyclic Jacobi eigensolver)
 *   A        = U^+ v_x U,  B = U^+ v_y U
 *   g_nm     = 1 / ((E_n - E_m)^2 + eta^2)
 *   sigma_j  = (2/N_k) sum_k sum_{n<m} (f_j(E_n) - f_j(E_m)) g_nm Im(A_nm B_mn)
 *
 * oracle_ahc_tensor evaluates the same band-pair sum for other pairs of
 * operators of the general response Eq. (1): the Hall tensor components
 * sigma_yz (v_y, v_z) and sigma_zx (v_z, v_x) next to sigma_xy, and the spin
 * Hall conductivity (spin current Js_x = (s_z v_x + v_x s_z)/2 with a diagonal
 * s_z, field along y).
 *
 * oracle_ahc_gf evaluates the Green's-function form the paper names for
 * systems with impurities (matrix inverses in place of eigenvalues; remark
 * after Eq. (3)), with a constant scattering rate gamma:
 *   G        = ((i (w + gamma) + mu) I - H(k))^{-1}      (explicit inverse)
 *   sigma_j  = (1/N_k) sum_k sum_l c_l Im{ Tr[G v_x G G v_y] - Tr[G v_y G G v_x] } / (2 pi)
 * at mu = E_F[j] and w = omega_l (> 0) for caller-given nodes and weights c_l
 * of a quadrature over the half line w > 0.  With gamma = 0 the w-integral
 * equals -sum_n theta(mu - E_n) Omega_n(eta = 0), i.e. Eqs. (2)-(3) at zero
 * temperature (residues of the poles at w = i (mu - E_n)).
 *
 * The reference gradient (oracle_ahc_grad) is derived in the design notes;
 * the paper has no adjoint.  It uses the divided-difference form of the
 * eigenvector term so that it stays finite through degeneracies.
 *
 * Layouts: t is complex128 [n_R][n][n] row-major (t[r][i][j] = t_ij(R_r)),
 * stored as interleaved (re, im) doubles; R is int32 [n_R][3].
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORACLE_MAX_SWEEPS 60
#define ORACLE_KCHUNK 4        /* k-points per fixed summation chunk of sigma */
#define ORACLE_GRAD_KCHUNK 64  /* k-points per gradient chunk (one G copy each) */

/* ------------------------------------------------------------------ */
/* Occupations (Eq. (3) uses a step; kT > 0 generalises to Fermi-Dirac) */
/* ------------------------------------------------------------------ */

static double occ(double e, double ef, double kT) {
    if (kT == 0.0) {
        if (e < ef) return 1.0;
        if (e > ef) return 0.0;
        return 0.5;
    }
    double u = (e - ef) / kT;
    if (u > 0.0) {
        double w = exp(-u);
        return w / (1.0 + w);
    }
    return 1.0 / (1.0 + exp(u));
}

/* d occ / dE; zero for the step (the Fermi-surface delta is dropped). */
static double docc(double e, double ef, double kT) {
    if (kT == 0.0) return 0.0;
    double u = (e - ef) / kT;
    double ch = cosh(0.5 * u);
    return -1.0 / (4.0 * kT * ch * ch);
}

static double bcast_g(double x, double eta) { return 1.0 / (x * x + eta * eta); }
static double bcast_dg(double x, double eta) {
    double d = x * x + eta * eta;
    return -2.0 * x / (d * d);
}

/* ------------------------------------------------------------------ */
/* Step 1: Bloch sums for H(k) and the velocities v_a = dH/dk_a.        */
/* ------------------------------------------------------------------ */

/* phase[r] = e^{i k.R_r} given as a per-R array; writes n*n complex each. */
static void build_hk(int n, int nR, const int* R, const cplx* t, const cplx* phase, cplx* H,
                     cplx* vx, cplx* vy) {
    size_t nn = (size_t)n * n;
    cplx* Ht = calloc(nn, sizeof(cplx));
    cplx* Xt = calloc(nn, sizeof(cplx));
    cplx* Yt = calloc(nn, sizeof(cplx));
    for (int r = 0; r < nR; ++r) {
        cplx ph = phase[r];
        cplx phx = I * (double)R[3 * r + 0] * ph;
        cplx phy = I * (double)R[3 * r + 1] * ph;
        const cplx* tr = t + (size_t)r * nn;
        for (size_t e = 0; e < nn; ++e) {
            Ht[e] += tr[e] * ph;
            Xt[e] += tr[e] * phx;
            Yt[e] += tr[e] * phy;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            size_t ij = (size_t)i * n + j, ji = (size_t)j * n + i;
            H[ij] = 0.5 * (Ht[ij] + conj(Ht[ji]));
            vx[ij] = 0.5 * (Xt[ij] + conj(Xt[ji]));
            vy[ij] = 0.5 * (Yt[ij] + conj(Yt[ji]));
        }
    free(Ht);
    free(Xt);
    free(Yt);
}

/* e^{i k.R} for the grid point (i0,i1,i2): each axis factor uses the exact
 * integer residue (i_a R_a mod N_a) so the angle is 2 pi m / N_a. */
static void grid_phases(int nR, const int* R, const int grid[3], long i0, long i1, long i2,
                        cplx* phase) {
    long idx[3] = {i0, i1, i2};
    for (int r = 0; r < nR; ++r) {
        cplx ph = 1.0;
        for (int a = 0; a < 3; ++a) {
            long N = grid[a];
            long m = ((idx[a] * (long)R[3 * r + a]) % N + N) % N;
            double ang = 2.0 * M_PI * (double)m / (double)N;
            ph *= cos(ang) + I * sin(ang);
        }
        phase[r] = ph;
    }
}

static void flat_to_ijk(long f, const int grid[3], long* i0, long* i1, long* i2) {
    *i0 = f % grid[0];
    long q = f / grid[0];
    *i1 = q % grid[1];
    *i2 = q / grid[1];
}

/* ------------------------------------------------------------------ */
/* Step 2: Hermitian eigensolver, cyclic (row-order) two-sided Jacobi.  */
/* ------------------------------------------------------------------ */

/* On entry A (n*n, row-major) is Hermitian; it is destroyed.  On exit E holds
 * the eigenvalues in ascending order and the columns of U the eigenvectors
 * (A_in U = U diag(E)).  Returns the number of sweeps, or -1 if the
 * off-diagonal mass failed to vanish in ORACLE_MAX_SWEEPS sweeps. */
static int jacobi_eigh(int n, cplx* A, double* E, cplx* U) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) U[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int i = 0; i < n; ++i) A[i * n + i] = creal(A[i * n + i]);
    int sweep = 0;
    int ok = 0;
    for (; sweep <= ORACLE_MAX_SWEEPS; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double a2 = creal(A[i * n + j]) * creal(A[i * n + j]) +
                            cimag(A[i * n + j]) * cimag(A[i * n + j]);
                tot += a2;
                if (i != j) off += a2;
            }
        if (off == 0.0 || off <= 1e-34 * tot) {
            ok = 1;
            break;
        }
        if (sweep == ORACLE_MAX_SWEEPS) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                cplx apq = A[p * n + q];
                double r = cabs(apq);
                if (r == 0.0) continue;
                cplx eph = apq / r; /* e^{i phi} */
                double app = creal(A[p * n + p]), aqq = creal(A[q * n + q]);
                double theta = (aqq - app) / (2.0 * r);
                double tn;
                if (fabs(theta) > 1e150)
                    tn = 0.5 / theta;
                else
                    tn = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(tn * tn + 1.0);
                double s = tn * c;
                /* J on the (p,q) plane: J = diag(1, e^{-i phi}) [[c, s], [-s, c]] */
                cplx Jpp = c, Jpq = s, Jqp = -s * conj(eph), Jqq = c * conj(eph);
                /* A <- A J (columns p, q) */
                for (int k = 0; k < n; ++k) {
                    cplx akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = akp * Jpp + akq * Jqp;
                    A[k * n + q] = akp * Jpq + akq * Jqq;
                }
                /* A <- J^+ A (rows p, q) */
                for (int k = 0; k < n; ++k) {
                    cplx apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = conj(Jpp) * apk + conj(Jqp) * aqk;
                    A[q * n + k] = conj(Jpq) * apk + conj(Jqq) * aqk;
                }
                A[p * n + q] = 0.0;
                A[q * n + p] = 0.0;
                A[p * n + p] = app - tn * r;
                A[q * n + q] = aqq + tn * r;
                /* U <- U J */
                for (int k = 0; k < n; ++k) {
                    cplx ukp = U[k * n + p], ukq = U[k * n + q];
                    U[k * n + p] = ukp * Jpp + ukq * Jqp;
                    U[k * n + q] = ukp * Jpq + ukq * Jqq;
                }
            }
    }
    for (int i = 0; i < n; ++i) E[i] = creal(A[i * n + i]);
    /* selection sort, ascending, swapping eigenvector columns alongside */
    for (int i = 0; i < n - 1; ++i) {
        int m = i;
        for (int j = i + 1; j < n; ++j)
            if (E[j] < E[m]) m = j;
        if (m != i) {
            double te = E[i];
            E[i] = E[m];
            E[m] = te;
            for (int k = 0; k < n; ++k) {
                cplx tu = U[k * n + i];
                U[k * n + i] = U[k * n + m];
                U[k * n + m] = tu;
            }
        }
    }
    return ok ? sweep : -1;
}

/* ------------------------------------------------------------------ */
/* Step 3: rotation into the eigenbasis, X' = U^+ X U.                  */
/* ------------------------------------------------------------------ */

static void rotate_in(int n, const cplx* U, const cplx* X, cplx* out) {
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            cplx s = 0.0;
            for (int i = 0; i < n; ++i) {
                cplx ui = conj(U[i * n + a]);
                if (ui == 0.0) continue;
                for (int j = 0; j < n; ++j) s += ui * X[i * n + j] * U[j * n + b];
            }
            out[a * n + b] = s;
        }
}

/* out = U X U^+ (the adjoint of rotate_in) */
static void rotate_out(int n, const cplx* U, const cplx* X, cplx* out) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            cplx s = 0.0;
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) s += U[i * n + a] * X[a * n + b] * conj(U[j * n + b]);
            out[i * n + j] = s;
        }
}

/* Steps 1-3 at one k given the per-R phases: E (ascending), U, A, B. */
static int eigen_velocities(int n, int nR, const int* R, const cplx* t, const cplx* phase,
                            double* E, cplx* U, cplx* A, cplx* B) {
    size_t nn = (size_t)n * n;
    cplx* H = malloc(nn * sizeof(cplx));
    cplx* vx = malloc(nn * sizeof(cplx));
    cplx* vy = malloc(nn * sizeof(cplx));
    build_hk(n, nR, R, t, phase, H, vx, vy);
    int sw = jacobi_eigh(n, H, E, U);
    rotate_in(n, U, vx, A);
    rotate_in(n, U, vy, B);
    free(H);
    free(vx);
    free(vy);
    return sw;
}

/* Neumaier-compensated accumulator */
typedef struct {
    double s, c;
} nsum;
static void nadd(nsum* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}
static double nval(const nsum* a) { return a->s + a->c; }

/* ------------------------------------------------------------------ */
/* Public entry points (called through ctypes from the test harness).   */
/* ------------------------------------------------------------------ */

int oracle_version(void) { return 1; }

/* H(k), v_x(k), v_y(k) at an arbitrary k (radians, cubic cell a = 1). */
int oracle_hk(int n, int nR, const int* R, const double* t, const double* k, double* H,
              double* vx, double* vy) {
    cplx* phase = malloc((size_t)nR * sizeof(cplx));
    for (int r = 0; r < nR; ++r) {
        double kr = k[0] * R[3 * r] + k[1] * R[3 * r + 1] + k[2] * R[3 * r + 2];
        phase[r] = cexp(I * kr);
    }
    build_hk(n, nR, R, (const cplx*)t, phase, (cplx*)H, (cplx*)vx, (cplx*)vy);
    free(phase);
    return 0;
}

/* Hermitian eigendecomposition of a user matrix (A is copied, not touched). */
int oracle_eigh(int n, const double* A_in, double* E, double* U) {
    size_t nn = (size_t)n * n;
    cplx* A = malloc(nn * sizeof(cplx));
    memcpy(A, A_in, nn * sizeof(cplx));
    int sw = jacobi_eigh(n, A, E, (cplx*)U);
    free(A);
    return sw;
}

/* Per-band quantities at an arbitrary k: E_n (ascending) and the broadened
 * Berry curvature Omega_n = -2 sum_{m != n} Im(A_nm B_mn) g_nm.  At eta = 0,
 * exactly degenerate pairs are skipped. */
int oracle_bands_k(int n, int nR, const int* R, const double* t, const double* k, double eta,
                   double* E, double* Omega) {
    size_t nn = (size_t)n * n;
    cplx* phase = malloc((size_t)nR * sizeof(cplx));
    for (int r = 0; r < nR; ++r) {
        double kr = k[0] * R[3 * r] + k[1] * R[3 * r + 1] + k[2] * R[3 * r + 2];
        phase[r] = cexp(I * kr);
    }
    cplx* U = malloc(nn * sizeof(cplx));
    cplx* A = malloc(nn * sizeof(cplx));
    cplx* B = malloc(nn * sizeof(cplx));
    int sw = eigen_velocities(n, nR, R, (const cplx*)t, phase, E, U, A, B);
    for (int a = 0; a < n; ++a) {
        double om = 0.0;
        for (int b = 0; b < n; ++b) {
            if (b == a) continue;
            double de = E[a] - E[b];
            if (eta == 0.0 && de == 0.0) continue;
            om += cimag(A[a * n + b] * B[b * n + a]) * bcast_g(de, eta);
        }
        Omega[a] = -2.0 * om;
    }
    free(phase);
    free(U);
    free(A);
    free(B);
    return sw < 0 ? -1 : 0;
}

/* sigma_xy[j] for every Fermi level, over the k-slab [k_begin, k_begin+k_count)
 * of the flat grid index, normalised by the FULL grid N_k so that disjoint
 * slabs add up.  sabs[j] (may be NULL) receives (1/N_k) sum of the absolute
 * pair terms, and sband[j] (may be NULL) (1/N_k) sum_k sum_n f_j(E_n)|Omega_n|,
 * the magnitude of the terms of the band form -(1/N_k) sum f Omega; they are
 * the scales against which rounding after cancellation is judged.  nthreads <= 0
 * uses the OpenMP default.  Returns 0, or -1 if some eigensolve did not
 * converge.  The k-sum is Neumaier-compensated in fixed chunks, so the result
 * does not depend on the thread count. */
int oracle_ahc(int n, int nR, const int* R, const double* t, const int* grid, long k_begin,
               long k_count, int nF, const double* EF, double eta, double kT, double* sigma,
               double* sabs, double* sband, int nthreads) {
    long Nk = (long)grid[0] * grid[1] * grid[2];
    long nchunk = (k_count + ORACLE_KCHUNK - 1) / ORACLE_KCHUNK;
    double* csum = calloc((size_t)nchunk * nF, sizeof(double));
    double* cabsum = calloc((size_t)nchunk * nF, sizeof(double));
    double* cband = calloc((size_t)nchunk * nF, sizeof(double));
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        size_t nn = (size_t)n * n;
        cplx* phase = malloc((size_t)nR * sizeof(cplx));
        cplx* U = malloc(nn * sizeof(cplx));
        cplx* A = malloc(nn * sizeof(cplx));
        cplx* B = malloc(nn * sizeof(cplx));
        double* E = malloc((size_t)n * sizeof(double));
        double* fo = malloc((size_t)n * nF * sizeof(double));
        nsum* acc = malloc((size_t)nF * sizeof(nsum));
        nsum* aab = malloc((size_t)nF * sizeof(nsum));
        nsum* abd = malloc((size_t)nF * sizeof(nsum));
        double* om = malloc((size_t)n * sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (long c = 0; c < nchunk; ++c) {
            for (int j = 0; j < nF; ++j) {
                acc[j].s = acc[j].c = 0.0;
                aab[j].s = aab[j].c = 0.0;
                abd[j].s = abd[j].c = 0.0;
            }
            long kb = k_begin + c * ORACLE_KCHUNK;
            long ke = kb + ORACLE_KCHUNK;
            if (ke > k_begin + k_count) ke = k_begin + k_count;
            for (long f = kb; f < ke; ++f) {
                long i0, i1, i2;
                flat_to_ijk(f, grid, &i0, &i1, &i2);
                grid_phases(nR, R, grid, i0, i1, i2, phase);
                if (eigen_velocities(n, nR, R, (const cplx*)t, phase, E, U, A, B) < 0) {
#pragma omp atomic write
                    bad = 1;
                }
                for (int a = 0; a < n; ++a)
                    for (int j = 0; j < nF; ++j) fo[a * nF + j] = occ(E[a], EF[j], kT);
                for (int a = 0; a < n; ++a)
                    for (int b = a + 1; b < n; ++b) {
                        double de = E[a] - E[b];
                        if (eta == 0.0 && de == 0.0) continue;
                        double w = 2.0 * bcast_g(de, eta) * cimag(A[a * n + b] * B[b * n + a]);
                        for (int j = 0; j < nF; ++j) {
                            double term = (fo[a * nF + j] - fo[b * nF + j]) * w;
                            nadd(&acc[j], term);
                            nadd(&aab[j], fabs(term));
                        }
                    }
                if (sband) {
                    for (int a = 0; a < n; ++a) {
                        double o = 0.0;
                        for (int b = 0; b < n; ++b) {
                            double de = E[a] - E[b];
                            if (b == a || (eta == 0.0 && de == 0.0)) continue;
                            o += cimag(A[a * n + b] * B[b * n + a]) * bcast_g(de, eta);
                        }
                        om[a] = fabs(2.0 * o);
                    }
                    for (int j = 0; j < nF; ++j)
                        for (int a = 0; a < n; ++a) nadd(&abd[j], fo[a * nF + j] * om[a]);
                }
            }
            for (int j = 0; j < nF; ++j) {
                csum[c * nF + j] = nval(&acc[j]);
                cabsum[c * nF + j] = nval(&aab[j]);
                cband[c * nF + j] = nval(&abd[j]);
            }
        }
        free(phase);
        free(U);
        free(A);
        free(B);
        free(E);
        free(fo);
        free(acc);
        free(aab);
        free(abd);
        free(om);
    }
    for (int j = 0; j < nF; ++j) {
        nsum s = {0.0, 0.0}, sa = {0.0, 0.0}, sb = {0.0, 0.0};
        for (long c = 0; c < nchunk; ++c) {
            nadd(&s, csum[c * nF + j]);
            nadd(&sa, cabsum[c * nF + j]);
            nadd(&sb, cband[c * nF + j]);
        }
        sigma[j] = nval(&s) / (double)Nk;
        if (sabs) sabs[j] = nval(&sa) / (double)Nk;
        if (sband) sband[j] = nval(&sb) / (double)Nk;
    }
    free(csum);
    free(cabsum);
    free(cband);
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* Other operator pairs of the general response (Eq. (1)): the Hall      */
/* tensor components xy, yz, zx and the spin Hall component.            */
/* ------------------------------------------------------------------ */

/* H(k) and the three velocities v_a = dH/dk_a (Hermitian parts), and, when
 * spin != NULL, the spin current Js_x = (S v_x + v_x S)/2 for the diagonal spin
 * operator S = diag(spin). */
static void build_hk3(int n, int nR, const int* R, const cplx* t, const cplx* phase,
                      const double* spin, cplx* H, cplx* v[3], cplx* js) {
    size_t nn = (size_t)n * n;
    cplx* Ht = calloc(nn, sizeof(cplx));
    cplx* Vt[3];
    for (int a = 0; a < 3; ++a) Vt[a] = calloc(nn, sizeof(cplx));
    for (int r = 0; r < nR; ++r) {
        const cplx* tr = t + (size_t)r * nn;
        cplx ph = phase[r];
        cplx pa[3];
        for (int a = 0; a < 3; ++a) pa[a] = I * (double)R[3 * r + a] * ph;
        for (size_t e = 0; e < nn; ++e) {
            Ht[e] += tr[e] * ph;
            for (int a = 0; a < 3; ++a) Vt[a][e] += tr[e] * pa[a];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            size_t ij = (size_t)i * n + j, ji = (size_t)j * n + i;
            H[ij] = 0.5 * (Ht[ij] + conj(Ht[ji]));
            for (int a = 0; a < 3; ++a) v[a][ij] = 0.5 * (Vt[a][ij] + conj(Vt[a][ji]));
        }
    if (spin)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                js[(size_t)i * n + j] = 0.5 * (spin[i] + spin[j]) * v[0][(size_t)i * n + j];
    free(Ht);
    for (int a = 0; a < 3; ++a) free(Vt[a]);
}

/* The four components, for every Fermi level j, over the k-slab (normalised by
 * the full grid):
 *   c = 0: sigma_xy (operators v_x, v_y)     c = 1: sigma_yz (v_y, v_z)
 *   c = 2: sigma_zx (v_z, v_x)               c = 3: spin Hall (Js_x, v_y), only
 *   when spin != NULL (else 0)
 * each in the pair form sigma_PQ = (2/N_k) sum_k sum_{n<m} (f_n - f_m) g_nm
 * Im(P'_nm Q'_mn) with P' = U^+ P U, Q' = U^+ Q U.  sigma and sabs are
 * [4][nF]; sabs (may be NULL) receives (1/N_k) sum of the absolute pair terms
 * and sband (may be NULL) (1/N_k) sum_k sum_n f_n |Omega^PQ_n| per component.
 * Returns 0, or -1 if an eigensolve did not converge. */
int oracle_ahc_tensor(int n, int nR, const int* R, const double* t, const int* grid, long k_begin,
                      long k_count, int nF, const double* EF, double eta, double kT,
                      const double* spin, double* sigma, double* sabs, double* sband,
                      int nthreads) {
    enum { NC = 4 };
    long Nk = (long)grid[0] * grid[1] * grid[2];
    long nchunk = (k_count + ORACLE_KCHUNK - 1) / ORACLE_KCHUNK;
    size_t per = (size_t)NC * nF;
    double* csum = calloc((size_t)nchunk * per, sizeof(double));
    double* cabsum = calloc((size_t)nchunk * per, sizeof(double));
    double* cband = calloc((size_t)nchunk * per, sizeof(double));
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        size_t nn = (size_t)n * n;
        cplx* phase = malloc((size_t)nR * sizeof(cplx));
        cplx* H = malloc(nn * sizeof(cplx));
        cplx* U = malloc(nn * sizeof(cplx));
        cplx* v[3];
        cplx* w[4]; /* rotated: v_x, v_y, v_z, Js_x */
        for (int a = 0; a < 3; ++a) v[a] = malloc(nn * sizeof(cplx));
        for (int a = 0; a < 4; ++a) w[a] = malloc(nn * sizeof(cplx));
        cplx* js = malloc(nn * sizeof(cplx));
        double* E = malloc((size_t)n * sizeof(double));
        double* fo = malloc((size_t)n * nF * sizeof(double));
        double* om = malloc((size_t)n * sizeof(double));
        nsum* acc = malloc(per * sizeof(nsum));
        nsum* aab = malloc(per * sizeof(nsum));
        nsum* abd = malloc(per * sizeof(nsum));
        const int pairs[NC][2] = {{0, 1}, {1, 2}, {2, 0}, {3, 1}};
#pragma omp for schedule(dynamic, 1)
        for (long c = 0; c < nchunk; ++c) {
            for (size_t q = 0; q < per; ++q) {
                acc[q].s = acc[q].c = 0.0;
                aab[q].s = aab[q].c = 0.0;
                abd[q].s = abd[q].c = 0.0;
            }
            long kb = k_begin + c * ORACLE_KCHUNK;
            long ke = kb + ORACLE_KCHUNK;
            if (ke > k_begin + k_count) ke = k_begin + k_count;
            for (long f = kb; f < ke; ++f) {
                long i0, i1, i2;
                flat_to_ijk(f, grid, &i0, &i1, &i2);
                grid_phases(nR, R, grid, i0, i1, i2, phase);
                build_hk3(n, nR, R, (const cplx*)t, phase, spin, H, v, js);
                if (jacobi_eigh(n, H, E, U) < 0) {
#pragma omp atomic write
                    bad = 1;
                }
                for (int a = 0; a < 3; ++a) rotate_in(n, U, v[a], w[a]);
                if (spin) rotate_in(n, U, js, w[3]);
                for (int a = 0; a < n; ++a)
                    for (int j = 0; j < nF; ++j) fo[a * nF + j] = occ(E[a], EF[j], kT);
                for (int comp = 0; comp < NC; ++comp) {
                    if (comp == 3 && !spin) continue;
                    const cplx* P = w[pairs[comp][0]];
                    const cplx* Q = w[pairs[comp][1]];
                    nsum* ac = acc + (size_t)comp * nF;
                    nsum* aa = aab + (size_t)comp * nF;
                    nsum* ab = abd + (size_t)comp * nF;
                    for (int a = 0; a < n; ++a)
                        for (int b = a + 1; b < n; ++b) {
                            double de = E[a] - E[b];
                            if (eta == 0.0 && de == 0.0) continue;
                            double wt = 2.0 * bcast_g(de, eta) * cimag(P[a * n + b] * Q[b * n + a]);
                            for (int j = 0; j < nF; ++j) {
                                double term = (fo[a * nF + j] - fo[b * nF + j]) * wt;
                                nadd(&ac[j], term);
                                nadd(&aa[j], fabs(term));
                            }
                        }
                    if (sband) {
                        for (int a = 0; a < n; ++a) {
                            double o = 0.0;
                            for (int b = 0; b < n; ++b) {
                                double de = E[a] - E[b];
                                if (b == a || (eta == 0.0 && de == 0.0)) continue;
                                o += cimag(P[a * n + b] * Q[b * n + a]) * bcast_g(de, eta);
                            }
                            om[a] = fabs(2.0 * o);
                        }
                        for (int j = 0; j < nF; ++j)
                            for (int a = 0; a < n; ++a) nadd(&ab[j], fo[a * nF + j] * om[a]);
                    }
                }
            }
            for (size_t q = 0; q < per; ++q) {
                csum[c * per + q] = nval(&acc[q]);
                cabsum[c * per + q] = nval(&aab[q]);
                cband[c * per + q] = nval(&abd[q]);
            }
        }
        free(phase);
        free(H);
        free(U);
        for (int a = 0; a < 3; ++a) free(v[a]);
        for (int a = 0; a < 4; ++a) free(w[a]);
        free(js);
        free(E);
        free(fo);
        free(om);
        free(acc);
        free(aab);
        free(abd);
    }
    for (size_t q = 0; q < per; ++q) {
        nsum s = {0.0, 0.0}, sa = {0.0, 0.0}, sb = {0.0, 0.0};
        for (long c = 0; c < nchunk; ++c) {
            nadd(&s, csum[c * per + q]);
            nadd(&sa, cabsum[c * per + q]);
            nadd(&sb, cband[c * per + q]);
        }
        sigma[q] = nval(&s) / (double)Nk;
        if (sabs) sabs[q] = nval(&sa) / (double)Nk;
        if (sband) sband[q] = nval(&sb) / (double)Nk;
    }
    free(csum);
    free(cabsum);
    free(cband);
    return bad ? -1 : 0;
}

/* Smallest and largest eigenvalue of H(k) over the slab of the grid. */
/* ------------------------------------------------------------------ */
/* Green's-function form (one explicit inverse per k, mu and node).     */
/* ------------------------------------------------------------------ */

/* Ainv = A^{-1} by Gauss-Jordan elimination on [A | I] with partial (row)
 * pivoting; A is destroyed.  Returns -1 for an exactly singular pivot. */
static int cinv(int n, cplx* A, cplx* Ainv) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ainv[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int p = 0; p < n; ++p) {
        int best = p;
        for (int i = p + 1; i < n; ++i)
            if (cabs(A[i * n + p]) > cabs(A[best * n + p])) best = i;
        if (A[best * n + p] == 0.0) return -1;
        if (best != p)
            for (int j = 0; j < n; ++j) {
                cplx x = A[p * n + j];
                A[p * n + j] = A[best * n + j];
                A[best * n + j] = x;
                x = Ainv[p * n + j];
                Ainv[p * n + j] = Ainv[best * n + j];
                Ainv[best * n + j] = x;
            }
        cplx d = 1.0 / A[p * n + p];
        for (int j = 0; j < n; ++j) {
            A[p * n + j] *= d;
            Ainv[p * n + j] *= d;
        }
        for (int i = 0; i < n; ++i) {
            if (i == p) continue;
            cplx f = A[i * n + p];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) {
                A[i * n + j] -= f * A[p * n + j];
                Ainv[i * n + j] -= f * Ainv[p * n + j];
            }
        }
    }
    return 0;
}

/* C = A B (n x n, row-major) */
static void cmatmul(int n, const cplx* A, const cplx* B, cplx* C) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            cplx s = 0.0;
            for (int k = 0; k < n; ++k) s += A[i * n + k] * B[k * n + j];
            C[i * n + j] = s;
        }
}

static cplx ctrace(int n, const cplx* A) {
    cplx s = 0.0;
    for (int i = 0; i < n; ++i) s += A[i * n + i];
    return s;
}

/* sigma[nF] as defined at the top of this file; sabs[nF] (optional) is the same
 * sum with |Tr[..]| + |Tr[..]| in place of Im{..}, a scale for rounding. */
int oracle_ahc_gf(int n, int nR, const int* R, const double* t, const int* grid, long k_begin,
                  long k_count, int nF, const double* EF, double gamma, int nw,
                  const double* omega, const double* weight, double* sigma, double* sabs,
                  int nthreads) {
    long Nk = (long)grid[0] * grid[1] * grid[2];
    long nchunk = (k_count + ORACLE_KCHUNK - 1) / ORACLE_KCHUNK;
    double* csum = calloc((size_t)nchunk * nF, sizeof(double));
    double* cabsum = calloc((size_t)nchunk * nF, sizeof(double));
    int bad = 0;
    const double inv2pi = 1.0 / (2.0 * M_PI);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        size_t nn = (size_t)n * n;
        cplx* phase = malloc((size_t)nR * sizeof(cplx));
        cplx* H = malloc(nn * sizeof(cplx));
        cplx* vx = malloc(nn * sizeof(cplx));
        cplx* vy = malloc(nn * sizeof(cplx));
        cplx* A = malloc(nn * sizeof(cplx));
        cplx* G = malloc(nn * sizeof(cplx));
        cplx* X = malloc(nn * sizeof(cplx));
        cplx* Y = malloc(nn * sizeof(cplx));
        cplx* M1 = malloc(nn * sizeof(cplx));
        cplx* M2 = malloc(nn * sizeof(cplx));
        nsum* acc = malloc((size_t)nF * sizeof(nsum));
        nsum* aab = malloc((size_t)nF * sizeof(nsum));
#pragma omp for schedule(dynamic, 1)
        for (long c = 0; c < nchunk; ++c) {
            for (int j = 0; j < nF; ++j) {
                acc[j].s = acc[j].c = 0.0;
                aab[j].s = aab[j].c = 0.0;
            }
            long kb = k_begin + c * ORACLE_KCHUNK;
            long ke = kb + ORACLE_KCHUNK;
            if (ke > k_begin + k_count) ke = k_begin + k_count;
            for (long f = kb; f < ke; ++f) {
                long i0, i1, i2;
                flat_to_ijk(f, grid, &i0, &i1, &i2);
                grid_phases(nR, R, grid, i0, i1, i2, phase);
                build_hk(n, nR, R, (const cplx*)t, phase, H, vx, vy);
                for (int j = 0; j < nF; ++j)
                    for (int l = 0; l < nw; ++l) {
                        const cplx z = I * (omega[l] + gamma) + EF[j];
                        for (int a = 0; a < n; ++a)
                            for (int b = 0; b < n; ++b)
                                A[a * n + b] = ((a == b) ? z : 0.0) - H[a * n + b];
                        if (cinv(n, A, G) != 0) {
#pragma omp atomic write
                            bad = 1;
                            continue;
                        }
                        /* Tr[G v_x G G v_y] = Tr[(G v_x G)(G v_y)], and x <-> y */
                        cmatmul(n, G, vx, X);
                        cmatmul(n, G, vy, Y);
                        cmatmul(n, X, G, M1);
                        cmatmul(n, M1, Y, M2);
                        const cplx t1 = ctrace(n, M2);
                        cmatmul(n, Y, G, M1);
                        cmatmul(n, M1, X, M2);
                        const cplx t2 = ctrace(n, M2);
                        nadd(&acc[j], weight[l] * cimag(t1 - t2) * inv2pi);
                        nadd(&aab[j], fabs(weight[l]) * (cabs(t1) + cabs(t2)) * inv2pi);
                    }
            }
            for (int j = 0; j < nF; ++j) {
                csum[c * nF + j] = nval(&acc[j]);
                cabsum[c * nF + j] = nval(&aab[j]);
            }
        }
        free(phase);
        free(H);
        free(vx);
        free(vy);
        free(A);
        free(G);
        free(X);
        free(Y);
        free(M1);
        free(M2);
        free(acc);
        free(aab);
    }
    for (int j = 0; j < nF; ++j) {
        nsum s = {0.0, 0.0}, sa = {0.0, 0.0};
        for (long c = 0; c < nchunk; ++c) {
            nadd(&s, csum[c * nF + j]);
            nadd(&sa, cabsum[c * nF + j]);
        }
        sigma[j] = nval(&s) / (double)Nk;
        if (sabs) sabs[j] = nval(&sa) / (double)Nk;
    }
    free(csum);
    free(cabsum);
    return bad ? -1 : 0;
}

int oracle_band_range(int n, int nR, const int* R, const double* t, const int* grid, double* emin,
                      double* emax, int nthreads) {
    long Nk = (long)grid[0] * grid[1] * grid[2];
    double lo = INFINITY, hi = -INFINITY;
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        size_t nn = (size_t)n * n;
        cplx* phase = malloc((size_t)nR * sizeof(cplx));
        cplx* H = malloc(nn * sizeof(cplx));
        cplx* vx = malloc(nn * sizeof(cplx));
        cplx* vy = malloc(nn * sizeof(cplx));
        cplx* U = malloc(nn * sizeof(cplx));
        double* E = malloc((size_t)n * sizeof(double));
        double tlo = INFINITY, thi = -INFINITY;
#pragma omp for schedule(dynamic, 4)
        for (long f = 0; f < Nk; ++f) {
            long i0, i1, i2;
            flat_to_ijk(f, grid, &i0, &i1, &i2);
            grid_phases(nR, R, grid, i0, i1, i2, phase);
            build_hk(n, nR, R, (const cplx*)t, phase, H, vx, vy);
            if (jacobi_eigh(n, H, E, U) < 0) {
#pragma omp atomic write
                bad = 1;
            }
            if (E[0] < tlo) tlo = E[0];
            if (E[n - 1] > thi) thi = E[n - 1];
        }
#pragma omp critical
        {
            if (tlo < lo) lo = tlo;
            if (thi > hi) hi = thi;
        }
        free(phase);
        free(H);
        free(vx);
        free(vy);
        free(U);
        free(E);
    }
    *emin = lo;
    *emax = hi;
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* Reference gradient of L = sum_j sbar_j sigma_j with respect to t(R).  */
/* ------------------------------------------------------------------ */

typedef struct {
    int nF;
    const double* EF;
    const double* sbar;
    double kT, eta;
} weights;

static double phi_of(const weights* w, double x) {
    double s = 0.0;
    for (int j = 0; j < w->nF; ++j) s += w->sbar[j] * occ(x, w->EF[j], w->kT);
    return s;
}
static double dphi_of(const weights* w, double x) {
    double s = 0.0;
    for (int j = 0; j < w->nF; ++j) s += w->sbar[j] * docc(x, w->EF[j], w->kT);
    return s;
}
/* K(x, y) = (phi(x) - phi(y)) g(x - y) and its x-derivative */
static double kern(const weights* w, double x, double y) {
    return (phi_of(w, x) - phi_of(w, y)) * bcast_g(x - y, w->eta);
}
static double dkern_dx(const weights* w, double x, double y) {
    return dphi_of(w, x) * bcast_g(x - y, w->eta) +
           (phi_of(w, x) - phi_of(w, y)) * bcast_dg(x - y, w->eta);
}

/* G[r] = dL/dRe t(R_r) + i dL/dIm t(R_r), complex128 [n_R][n][n], for the
 * slab of the grid (normalised by the full N_k, like oracle_ahc).  Every
 * entry of t is an independent parameter (the forward projects H onto its
 * Hermitian part).  mode 0: divided-difference form for the eigenvector term
 * (finite through degeneracies); mode 1: the plain commutator form
 * X_mn / (E_m - E_n) with a separate eigenvalue term, valid only when no two
 * eigenvalues coincide (used to cross-check mode 0).  Requires eta > 0. */
int oracle_ahc_grad(int n, int nR, const int* R, const double* t, const int* grid, long k_begin,
                    long k_count, int nF, const double* EF, double eta, double kT,
                    const double* sbar, double* G_out, int mode, int nthreads) {
    if (!(eta > 0.0)) return -2;
    long Nk = (long)grid[0] * grid[1] * grid[2];
    size_t nn = (size_t)n * n;
    size_t gsz = (size_t)nR * nn;
    long nchunk = (k_count + ORACLE_GRAD_KCHUNK - 1) / ORACLE_GRAD_KCHUNK;
    cplx* Gc = calloc((size_t)nchunk * gsz, sizeof(cplx));
    weights W = {nF, EF, sbar, kT, eta};
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        cplx* phase = malloc((size_t)nR * sizeof(cplx));
        cplx* U = malloc(nn * sizeof(cplx));
        cplx* A = malloc(nn * sizeof(cplx));
        cplx* B = malloc(nn * sizeof(cplx));
        cplx* Ab = malloc(nn * sizeof(cplx));
        cplx* Bb = malloc(nn * sizeof(cplx));
        cplx* Hb = malloc(nn * sizeof(cplx));
        cplx* Hbo = malloc(nn * sizeof(cplx));
        cplx* Vxo = malloc(nn * sizeof(cplx));
        cplx* Vyo = malloc(nn * sizeof(cplx));
        double* E = malloc((size_t)n * sizeof(double));
        const double inv = 1.0 / (double)Nk;
#pragma omp for schedule(dynamic, 1)
        for (long c = 0; c < nchunk; ++c) {
            cplx* Gk = Gc + (size_t)c * gsz;
            long kb = k_begin + c * ORACLE_GRAD_KCHUNK;
            long ke = kb + ORACLE_GRAD_KCHUNK;
            if (ke > k_begin + k_count) ke = k_begin + k_count;
            for (long f = kb; f < ke; ++f) {
                long i0, i1, i2;
                flat_to_ijk(f, grid, &i0, &i1, &i2);
                grid_phases(nR, R, grid, i0, i1, i2, phase);
                if (eigen_velocities(n, nR, R, (const cplx*)t, phase, E, U, A, B) < 0) {
#pragma omp atomic write
                    bad = 1;
                }
                double spread = E[n - 1] - E[0];
                double delta = 1e-8 * (spread > 0.0 ? spread : 1.0);
                /* cotangents of the eigenbasis velocities */
                for (int m = 0; m < n; ++m)
                    for (int q = 0; q < n; ++q) {
                        double K = (m == q) ? 0.0 : kern(&W, E[m], E[q]);
                        Ab[m * n + q] = I * inv * K * B[m * n + q];
                        Bb[m * n + q] = -I * inv * K * A[m * n + q];
                    }
                if (mode == 0) {
                    for (int m = 0; m < n; ++m)
                        for (int q = 0; q < n; ++q) {
                            cplx s = 0.0;
                            double de = E[m] - E[q];
                            for (int p = 0; p < n; ++p) {
                                double D;
                                if (fabs(de) < delta)
                                    D = dkern_dx(&W, 0.5 * (E[m] + E[q]), E[p]);
                                else
                                    D = (kern(&W, E[m], E[p]) - kern(&W, E[q], E[p])) / de;
                                s += D * (B[m * n + p] * A[p * n + q] - A[m * n + p] * B[p * n + q]);
                            }
                            Hb[m * n + q] = I * inv * s;
                        }
                } else {
                    /* X = [Ab, A] + [Bb, B];  Y_mq = X_mq / (E_m - E_q) off the diagonal,
                     * and the eigenvalue cotangent on it. */
                    for (int m = 0; m < n; ++m)
                        for (int q = 0; q < n; ++q) {
                            cplx x = 0.0;
                            for (int p = 0; p < n; ++p)
                                x += Ab[m * n + p] * A[p * n + q] - A[m * n + p] * Ab[p * n + q] +
                                     Bb[m * n + p] * B[p * n + q] - B[m * n + p] * Bb[p * n + q];
                            if (m == q) {
                                double eb = 0.0;
                                for (int p = 0; p < n; ++p) {
                                    if (p == m) continue;
                                    double qmp = cimag(A[m * n + p] * B[p * n + m]);
                                    eb += qmp * dkern_dx(&W, E[m], E[p]);
                                }
                                Hb[m * n + m] = 2.0 * inv * eb;
                            } else {
                                Hb[m * n + q] = x / (E[m] - E[q]);
                            }
                        }
                }
                rotate_out(n, U, Hb, Hbo);
                rotate_out(n, U, Ab, Vxo);
                rotate_out(n, U, Bb, Vyo);
                for (int r = 0; r < nR; ++r) {
                    cplx cph = conj(phase[r]);
                    double Rx = R[3 * r], Ry = R[3 * r + 1];
                    cplx* Gr = Gk + (size_t)r * nn;
                    for (size_t e = 0; e < nn; ++e)
                        Gr[e] += cph * (Hbo[e] - I * Rx * Vxo[e] - I * Ry * Vyo[e]);
                }
            }
        }
        free(phase);
        free(U);
        free(A);
        free(B);
        free(Ab);
        free(Bb);
        free(Hb);
        free(Hbo);
        free(Vxo);
        free(Vyo);
        free(E);
    }
    cplx* G = (cplx*)G_out;
    for (size_t e = 0; e < gsz; ++e) {
        cplx s = 0.0;
        for (long c = 0; c < nchunk; ++c) s += Gc[(size_t)c * gsz + e];
        G[e] = s;
    }
    free(Gc);
    return bad ? -1 : 0;
}
