// kubo_device.hip -- gfx950 kernels of the Kubo-formula Hall-conductivity path.
//
// Forward pipeline for one batch of k-points (paper: the four per-k steps of
// the baseline listing, batched as in its Eq. (4)):
//   k_hermproj   t'(R) = (t(R) + t(-R)^+)/2, so that H(k) = sum_R t'(R) e^{ik.R}
//                is the Hermitian part of the Bloch sum.
//   k_pencil     sum factorisation of the Bloch sum over one kx pencil:
//                T_rho  = sum_{R: R_x = rho} t'(R) e^{i(k1 R_y + k2 R_z)}
//                Ty_rho = sum_{R: R_x = rho} i R_y t'(R) e^{i(k1 R_y + k2 R_z)}
//   k_forward    per k-point: H = sum_rho e^{i k0 rho} T_rho,
//                v_x = sum_rho i rho e^{i k0 rho} T_rho, v_y = sum_rho e^{i k0 rho} Ty_rho
//                (step 1); parallel-order two-sided Jacobi eigensolver (step 2);
//                A = U^+ v_x U, B = U^+ v_y U (step 3); Berry curvature
//                Omega_n = -2 sum_m Im(A_nm B_mn) g(E_n - E_m) and the Fermi-weighted
//                sums s_j = sum_n f_j(E_n) Omega_n accumulated per k-block (step 4).
//   k_reduce     sigma_j = -(1/N_k) sum over the model's k-blocks, fixed tree order.
// All arithmetic is FP64.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kubo_cplx.h"
#include "kubo_internal.h"
#include "kubo_launch.h"

namespace kubo {

// Workgroup-wide sum of two doubles (NT threads, LDS scratch of 2*NT/64 doubles).
template <int NT>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    constexpr int NW = NT / 64;
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        red[w] = a;
        red[NW + w] = b;
    }
    __syncthreads();
    a = 0.0;
    b = 0.0;
    for (int i = 0; i < NW; ++i) {
        a += red[i];
        b += red[NW + i];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// k_clear: zero the status word (a kernel, not a memset, so graphs replay it)
// ---------------------------------------------------------------------------
__global__ void k_clear_status(unsigned* status) {
    if (threadIdx.x == 0 && blockIdx.x == 0) status[0] = 0u;
}

__global__ void k_zero(double* p, long long count) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// k_hermproj: t'(R) = (t(R) + t(-R)^+)/2 over all models of the plan
// ---------------------------------------------------------------------------
__global__ void k_hermproj(Tables tb, int n_models, long long total, const double2* __restrict__ t,
                           double2* __restrict__ tp) {
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; e < total; e += stride) {
        int lo = 0, hi = n_models - 1;
        while (lo < hi) {  // last model with t_off <= e
            int mid = (lo + hi + 1) >> 1;
            if (tb.models[mid].t_off <= e)
                lo = mid;
            else
                hi = mid - 1;
        }
        const ModelDev& md = tb.models[lo];
        long long loc = e - md.t_off;
        int n = md.n;
        long long nn = (long long)n * n;
        int r = (int)(loc / nn);
        int ij = (int)(loc - (long long)r * nn);
        int i = ij / n, j = ij - (ij / n) * n;
        int rn = tb.negr[md.neg_first + r];
        double2 a = t[md.t_off + loc];
        double2 b = t[md.t_off + (long long)rn * nn + (long long)j * n + i];
        tp[md.t_off + loc] = c_make(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    }
}

// ---------------------------------------------------------------------------
// k_pencil: per (model, i1, i2) the rho-resolved partial Bloch sums
// ---------------------------------------------------------------------------
constexpr int kPencilThreads = 256;
constexpr int kPencilPhaseTile = 512;

__global__ __launch_bounds__(kPencilThreads) void k_pencil(Tables tb, int item_begin,
                                                           const double2* __restrict__ tp,
                                                           double2* __restrict__ tbuf) {
    __shared__ double2 sph[kPencilPhaseTile];
    const PencilItem it = tb.pencils[item_begin + blockIdx.x];
    const ModelDev md = tb.models[it.model];
    const int n = md.n;
    const long long nn = (long long)n * n;
    double2* T0 = tbuf + it.tbuf_off;
    double2* T1 = T0 + (long long)md.nR0 * nn;
    const int* gstart = tb.grp_start + md.gs_first;
    for (int rho = 0; rho < md.nR0; ++rho) {
        const int g0 = gstart[rho], g1 = gstart[rho + 1];
        // elements handled by this thread: e = tid, tid + NT, ...  (accumulate over R tiles)
        for (long long e0 = 0; e0 < nn; e0 += kPencilThreads * 4) {
            double2 a0[4], a1[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) a0[u] = a1[u] = c_make(0.0, 0.0);
            for (int gt = g0; gt < g1; gt += kPencilPhaseTile) {
                const int gcount = min(kPencilPhaseTile, g1 - gt);
                __syncthreads();
                for (int g = threadIdx.x; g < gcount; g += kPencilThreads) {
                    int gi = md.grp_first + gt + g;
                    sph[g] = unit_phase2((long long)it.i1 * tb.grp_R1[gi], md.N1,
                                         (long long)it.i2 * tb.grp_R2[gi], md.N2);
                }
                __syncthreads();
                for (int g = 0; g < gcount; ++g) {
                    const int gi = md.grp_first + gt + g;
                    const int r = tb.grp_r[gi];
                    const double ry = (double)tb.grp_R1[gi];
                    const double2 ph = sph[g];
                    const double2 phy = c_i(c_scale(ry, ph));
                    const double2* tr = tp + md.t_off + (long long)r * nn;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        long long e = e0 + threadIdx.x + (long long)u * kPencilThreads;
                        if (e < nn) {
                            double2 v = tr[e];
                            a0[u] = c_fma(v, ph, a0[u]);
                            a1[u] = c_fma(v, phy, a1[u]);
                        }
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                long long e = e0 + threadIdx.x + (long long)u * kPencilThreads;
                if (e < nn) {
                    T0[(long long)rho * nn + e] = a0[u];
                    T1[(long long)rho * nn + e] = a1[u];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Eigensolver: parallel-order (round-robin) two-sided Jacobi in LDS.
//
// The nE = n + (n odd) indices are split into nE/2 disjoint pairs per round;
// nE - 1 rounds visit every pair once (one sweep).  Each round computes the
// nE/2 rotations, then every 2x2 block (rows of pair a, columns of pair b)
// is updated as J_a^+ X J_b, so each element of A is read and written once.
// ---------------------------------------------------------------------------
template <int NP>
struct JacobiLds {
    int p[NP / 2], q[NP / 2];
    double c[NP / 2], s[NP / 2];
    double2 eb[NP / 2];   // e^{-i phi}
    double dp[NP / 2], dq[NP / 2];
};

__device__ __forceinline__ void rr_pair(int r, int a, int nE, int& p, int& q) {
    const int m = nE - 1;
    int x, y;
    if (a == 0) {
        x = r;
        y = m;
    } else {
        x = (r + a) % m;
        y = (r - a + m) % m;
    }
    p = min(x, y);
    q = max(x, y);
}

// A (LD stride, n valid, zero-padded to nE) -> diagonal; V (LD) <- eigenvectors.
// Returns the number of sweeps performed, or -1 if the cap was reached.
template <int NP, int NT, int LD>
__device__ int jacobi_eigh(double2* A, double2* V, int n, int max_sweeps, JacobiLds<NP>& J,
                           double* red) {
    const int nE = n + (n & 1);
    const int P = nE / 2;
    for (int e = threadIdx.x; e < nE * nE; e += NT) {
        int i = e / nE, j = e - (e / nE) * nE;
        V[i * LD + j] = c_make(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    int sweep = 0;
    for (;; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int e = threadIdx.x; e < n * n; e += NT) {
            int i = e / n, j = e - (e / n) * n;
            double2 v = A[i * LD + j];
            double a2 = v.x * v.x + v.y * v.y;
            tot += a2;
            if (i != j) off += a2;
        }
        block_sum2<NT>(off, tot, red);
        if (off == 0.0 || off <= 1e-34 * tot) return sweep;
        if (sweep >= max_sweeps) return -1;
        for (int r = 0; r < nE - 1; ++r) {
            for (int a = threadIdx.x; a < P; a += NT) {
                int p, q;
                rr_pair(r, a, nE, p, q);
                J.p[a] = p;
                J.q[a] = q;
                double c = 1.0, s = 0.0;
                double2 eb = c_make(1.0, 0.0);
                double app = A[p * LD + p].x, aqq = A[q * LD + q].x;
                if (q < n) {
                    double2 apq = A[p * LD + q];
                    double rr = hypot(apq.x, apq.y);
                    if (rr > 0.0) {
                        eb = c_make(apq.x / rr, -apq.y / rr);
                        double theta = (aqq - app) / (2.0 * rr);
                        double t;
                        if (fabs(theta) > 1e150)
                            t = 0.5 / theta;
                        else
                            t = copysign(1.0, theta) / (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                        app -= t * rr;
                        aqq += t * rr;
                    }
                }
                J.c[a] = c;
                J.s[a] = s;
                J.eb[a] = eb;
                J.dp[a] = app;
                J.dq[a] = aqq;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < P * P; e += NT) {
                const int a = e / P, b = e - (e / P) * P;
                const int pa = J.p[a], qa = J.q[a], pb = J.p[b], qb = J.q[b];
                if (a == b) {
                    A[pa * LD + pa] = c_make(J.dp[a], 0.0);
                    A[qa * LD + qa] = c_make(J.dq[a], 0.0);
                    A[pa * LD + qa] = c_make(0.0, 0.0);
                    A[qa * LD + pa] = c_make(0.0, 0.0);
                    continue;
                }
                const double cb = J.c[b], sb = J.s[b];
                const double2 ebb = J.eb[b];
                const double ca = J.c[a], sa = J.s[a];
                const double2 ea = c_conj(J.eb[a]);  // e^{+i phi_a}
                const double2 x00 = A[pa * LD + pb], x01 = A[pa * LD + qb];
                const double2 x10 = A[qa * LD + pb], x11 = A[qa * LD + qb];
                // Y = X J_b with J_b = [[c, s], [-s eb, c eb]]
                const double2 x01e = c_mul(x01, ebb), x11e = c_mul(x11, ebb);
                const double2 y00 = c_sub(c_scale(cb, x00), c_scale(sb, x01e));
                const double2 y01 = c_add(c_scale(sb, x00), c_scale(cb, x01e));
                const double2 y10 = c_sub(c_scale(cb, x10), c_scale(sb, x11e));
                const double2 y11 = c_add(c_scale(sb, x10), c_scale(cb, x11e));
                // Z = J_a^+ Y with J_a^+ = [[c, -s e], [s, c e]]
                const double2 y10e = c_mul(y10, ea), y11e = c_mul(y11, ea);
                A[pa * LD + pb] = c_sub(c_scale(ca, y00), c_scale(sa, y10e));
                A[pa * LD + qb] = c_sub(c_scale(ca, y01), c_scale(sa, y11e));
                A[qa * LD + pb] = c_add(c_scale(sa, y00), c_scale(ca, y10e));
                A[qa * LD + qb] = c_add(c_scale(sa, y01), c_scale(ca, y11e));
            }
            for (int e = threadIdx.x; e < n * P; e += NT) {
                const int i = e / P, a = e - (e / P) * P;
                const int pa = J.p[a], qa = J.q[a];
                const double ca = J.c[a], sa = J.s[a];
                const double2 eb = J.eb[a];
                const double2 vp = V[i * LD + pa];
                const double2 vqe = c_mul(V[i * LD + qa], eb);
                V[i * LD + pa] = c_sub(c_scale(ca, vp), c_scale(sa, vqe));
                V[i * LD + qa] = c_add(c_scale(sa, vp), c_scale(ca, vqe));
            }
            __syncthreads();
        }
    }
}

// C = X * Y (n x n, strides LD), or C = X^+ * Y when ADJ_X.
template <int NT, int LD, bool ADJ_X>
__device__ __forceinline__ void gemm_n(double2* __restrict__ C, const double2* __restrict__ X,
                                       const double2* __restrict__ Y, int n) {
    for (int e = threadIdx.x; e < n * n; e += NT) {
        const int i = e / n, j = e - (e / n) * n;
        double2 acc = c_make(0.0, 0.0);
        if (ADJ_X) {
            for (int l = 0; l < n; ++l) acc = c_fmac(X[l * LD + i], Y[l * LD + j], acc);
        } else {
            for (int l = 0; l < n; ++l) acc = c_fma(X[i * LD + l], Y[l * LD + j], acc);
        }
        C[i * LD + j] = acc;
    }
}

// C = X * Y^+ (n x n, strides LD).
template <int NT, int LD>
__device__ __forceinline__ void gemm_n_adjy(double2* __restrict__ C, const double2* __restrict__ X,
                                            const double2* __restrict__ Y, int n) {
    for (int e = threadIdx.x; e < n * n; e += NT) {
        const int i = e / n, j = e - (e / n) * n;
        double2 acc = c_make(0.0, 0.0);
        for (int l = 0; l < n; ++l) acc = c_fma(X[i * LD + l], c_conj(Y[j * LD + l]), acc);
        C[i * LD + j] = acc;
    }
}

// Steps 1-3 at one k-point (i0 along the pencil whose partial sums are T0/T1):
//   H = sum_rho e^{i k0 rho} T0_rho, v_x = sum_rho i rho e^{i k0 rho} T0_rho,
//   v_y = sum_rho e^{i k0 rho} T1_rho; Jacobi eigendecomposition H = U E U^+;
//   on return E[0..n), V = U, X = U^+ v_x U, Y = U^+ v_y U (A is scratch).
template <int NP, int NT, int LD>
__device__ void eigen_at_k(const ModelDev& md, const double2* __restrict__ T0,
                           const double2* __restrict__ T1, const int* __restrict__ r0, int i0,
                           int max_sweeps, unsigned* status, double2* A, double2* V, double2* X,
                           double2* Y, double* E, double2* ph, JacobiLds<NP>& J, double* red) {
    const int n = md.n;
    const int nE = n + (n & 1);
    const long long nn = (long long)n * n;
    if (threadIdx.x < md.nR0) ph[threadIdx.x] = unit_phase((long long)i0 * r0[threadIdx.x], md.N0);
    __syncthreads();
    // step 1: upper triangle computed, lower mirrored, diagonal real, padding zero
    for (int e = threadIdx.x; e < nE * nE; e += NT) {
        const int i = e / nE, j = e - (e / nE) * nE;
        if (i > j) continue;
        double2 h = c_make(0.0, 0.0), x = h, y = h;
        if (j < n) {
            for (int rho = 0; rho < md.nR0; ++rho) {
                const double2 p = ph[rho];
                const double2 t0 = T0[(long long)rho * nn + i * n + j];
                const double2 t1 = T1[(long long)rho * nn + i * n + j];
                const double2 p0 = c_mul(t0, p);
                h = c_add(h, p0);
                x = c_add(x, c_scale((double)r0[rho], c_i(p0)));
                y = c_fma(t1, p, y);
            }
        }
        if (i == j) {
            h.y = 0.0;
            x.y = 0.0;
            y.y = 0.0;
        }
        A[i * LD + j] = h;
        A[j * LD + i] = c_conj(h);
        X[i * LD + j] = x;
        X[j * LD + i] = c_conj(x);
        Y[i * LD + j] = y;
        Y[j * LD + i] = c_conj(y);
    }
    __syncthreads();
    // step 2: eigendecomposition
    const int sw = jacobi_eigh<NP, NT, LD>(A, V, n, max_sweeps, J, red);
    if (sw < 0 && threadIdx.x == 0) atomicOr(status, kStatNoConv);
    for (int i = threadIdx.x; i < n; i += NT) E[i] = A[i * LD + i].x;
    __syncthreads();
    // step 3: X <- U^+ v_x U, Y <- U^+ v_y U (A is the scratch product)
    gemm_n<NT, LD, false>(A, X, V, n);
    __syncthreads();
    gemm_n<NT, LD, true>(X, V, A, n);
    __syncthreads();
    gemm_n<NT, LD, false>(A, Y, V, n);
    __syncthreads();
    gemm_n<NT, LD, true>(Y, V, A, n);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// k_forward: steps 1-4 for a list of k-blocks (persistent over the list)
// ---------------------------------------------------------------------------
struct FwdArgs {
    Tables tb;
    const double2* tbuf;   // chunk T region
    const double* e_fermi; // [models][nF]
    double* partial;       // [slots][nF]
    unsigned* status;
    double eta, kT;
    int nF;
    int max_sweeps;
    int item_begin, item_count;
};

template <int NP, int NT>
struct FwdLds {
    static constexpr int LD = NP + 1;
    double2 A[NP * LD];
    double2 V[NP * LD];
    double2 X[NP * LD];
    double2 Y[NP * LD];
    JacobiLds<NP> J;
    double E[NP];
    double Om[NP];
    double2 ph[16];
    double red[2 * (NT / 64)];
};

template <int NP, int NT>
__global__ __launch_bounds__(NT) void k_forward(FwdArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    FwdLds<NP, NT>& S = *reinterpret_cast<FwdLds<NP, NT>*>(smem_raw);
    constexpr int LD = FwdLds<NP, NT>::LD;
    const double eta2 = a.eta * a.eta;
    for (int item = blockIdx.x; item < a.item_count; item += gridDim.x) {
        const BlockItem it = a.tb.blocks[a.item_begin + item];
        const ModelDev md = a.tb.models[it.model];
        const int n = md.n;
        const long long nn = (long long)n * n;
        const double2* T0 = a.tbuf + it.tbuf_off;
        const double2* T1 = T0 + (long long)md.nR0 * nn;
        const int* r0 = a.tb.r0val + md.r0_first;
        const double* ef = a.e_fermi + md.f_off;
        double* part = a.partial + (long long)it.slot * a.nF;
        for (int kk = 0; kk < it.count; ++kk) {
            eigen_at_k<NP, NT, LD>(md, T0, T1, r0, it.i0 + kk, a.max_sweeps, a.status, S.A, S.V,
                                   S.X, S.Y, S.E, S.ph, S.J, S.red);
            // step 4a: Omega_n = -2 sum_{m != n} Im(A_nm B_mn) g(E_n - E_m)
            for (int b = threadIdx.x; b < n; b += NT) {
                double om = 0.0;
                const double eb = S.E[b];
                for (int m = 0; m < n; ++m) {
                    if (m == b) continue;
                    const double de = eb - S.E[m];
                    const double den = de * de + eta2;
                    if (den == 0.0) continue;
                    const double2 x = S.X[b * LD + m], y = S.Y[m * LD + b];
                    om += (x.x * y.y + x.y * y.x) / den;
                }
                S.Om[b] = -2.0 * om;
            }
            __syncthreads();
            // step 4b: s_j = sum_n f_j(E_n) Omega_n, accumulated over the block in fixed order
            for (int j = threadIdx.x; j < a.nF; j += NT) {
                const double efj = ef[j];
                double s = 0.0;
                for (int b = 0; b < n; ++b) s += occupation(S.E[b], efj, a.kT) * S.Om[b];
                if (!isfinite(s)) atomicOr(a.status, kStatNonFinite);
                part[j] = (kk == 0) ? s : part[j] + s;
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// k_adjoint: reverse mode of steps 1-4 for a list of k-blocks.
//
// For L = sum_j sbar_j sigma_j the per-k contribution is
//   L_k = (1/N_k) sum_{m != n} K_mn Im(A_mn B_nm),  K_mn = (phi_m - phi_n) g(E_m - E_n),
//   phi(E) = sum_j sbar_j f_j(E).
// Cotangents in the eigenbasis (complex-autograd convention):
//   Abar = (i/N_k) K o B,  Bbar = -(i/N_k) K o A,
//   Hbar' = diag(Ebar) + Y with Y_mn = X_mn / (E_m - E_n), X = [Abar, A] + [Bbar, B];
// X_mn = (i/N_k) sum_p (K_mp - K_np)(B_mp A_pn - A_mp B_pn) vanishes with E_m - E_n, so
// for near-degenerate pairs (and the diagonal, where it gives Ebar) the quotient is
// replaced by its limit: the x-derivative of K(x, E_p) at the mid point.
// Back in the orbital basis: Hbar = U Hbar' U^+, vbar_x = U Abar U^+, vbar_y = U Bbar U^+.
// The transposed Bloch sum is split like the forward one: per k-block the pencil partials
//   PH_rho = sum_k e^{-i k0 rho} (Hbar - i rho vbar_x),  PY_rho = sum_k e^{-i k0 rho} vbar_y
// are written to the workspace; k_gacc finishes the sum over R_y, R_z.
// ---------------------------------------------------------------------------
struct AdjArgs {
    Tables tb;
    const double2* tbuf;
    double2* pbuf;
    const double* e_fermi;
    const double* sbar;
    unsigned* status;
    double eta, kT;
    int nF;
    int max_sweeps;
    int item_begin, item_count;
};

template <int NP, int NT>
struct AdjLds {
    static constexpr int LD = NP + 1;
    double2 A[NP * LD];  // eigensolver scratch, then Hbar' and Hbar
    double2 V[NP * LD];  // U
    double2 X[NP * LD];  // A = U^+ v_x U, then vbar_y
    double2 Y[NP * LD];  // B = U^+ v_y U, then vbar_x
    double2 T[NP * LD];  // product scratch
    double K[NP * LD];
    JacobiLds<NP> J;
    double E[NP];
    double phi[NP];
    double dphi[NP];
    double2 ph[16];
    double red[2 * (NT / 64)];
};

// phi(x) = sum_j sbar_j f_j(x) and its derivative
__device__ __forceinline__ void phi_at(double x, const double* __restrict__ ef,
                                       const double* __restrict__ sb, int nF, double kT,
                                       double& phi, double& dphi) {
    double p = 0.0, d = 0.0;
    for (int j = 0; j < nF; ++j) {
        p += sb[j] * occupation(x, ef[j], kT);
        if (kT > 0.0) {
            const double ch = cosh(0.5 * (x - ef[j]) / kT);
            d -= sb[j] / (4.0 * kT * ch * ch);
        }
    }
    phi = p;
    dphi = d;
}

template <int NP, int NT>
__global__ __launch_bounds__(NT) void k_adjoint(AdjArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    AdjLds<NP, NT>& S = *reinterpret_cast<AdjLds<NP, NT>*>(smem_raw);
    constexpr int LD = AdjLds<NP, NT>::LD;
    const double eta2 = a.eta * a.eta;
    const double scale = (a.kT > 0.0) ? fmin(a.eta, a.kT) : a.eta;
    const double delta = 1e-5 * scale;  // below it the divided difference uses its limit
    for (int item = blockIdx.x; item < a.item_count; item += gridDim.x) {
        const BlockItem it = a.tb.blocks[a.item_begin + item];
        const ModelDev md = a.tb.models[it.model];
        const int n = md.n;
        const long long nn = (long long)n * n;
        const double2* T0 = a.tbuf + it.tbuf_off;
        const double2* T1 = T0 + (long long)md.nR0 * nn;
        double2* PH = a.pbuf + it.pbuf_off;
        double2* PY = PH + (long long)md.nR0 * nn;
        const int* r0 = a.tb.r0val + md.r0_first;
        const double* ef = a.e_fermi + md.f_off;
        const double* sb = a.sbar + md.f_off;
        const double invN = 1.0 / (double)md.Nk;
        for (int kk = 0; kk < it.count; ++kk) {
            const int i0 = it.i0 + kk;
            eigen_at_k<NP, NT, LD>(md, T0, T1, r0, i0, a.max_sweeps, a.status, S.A, S.V, S.X,
                                   S.Y, S.E, S.ph, S.J, S.red);
            for (int b = threadIdx.x; b < n; b += NT) {
                double p, d;
                phi_at(S.E[b], ef, sb, a.nF, a.kT, p, d);
                S.phi[b] = p;
                S.dphi[b] = d;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < n * n; e += NT) {
                const int m = e / n, q = e - (e / n) * n;
                double k = 0.0;
                if (m != q) {
                    const double de = S.E[m] - S.E[q];
                    k = (S.phi[m] - S.phi[q]) / (de * de + eta2);
                }
                S.K[m * LD + q] = k;
            }
            __syncthreads();
            // Hbar' in the eigenbasis (into A)
            for (int e = threadIdx.x; e < n * n; e += NT) {
                const int m = e / n, q = e - (e / n) * n;
                const double de = S.E[m] - S.E[q];
                double2 acc = c_make(0.0, 0.0);
                if (m != q && fabs(de) >= delta) {
                    for (int p = 0; p < n; ++p) {
                        const double w = S.K[m * LD + p] - S.K[q * LD + p];
                        // B_mp A_pq - A_mp B_pq
                        double2 z = c_mul(S.Y[m * LD + p], S.X[p * LD + q]);
                        z = c_sub(z, c_mul(S.X[m * LD + p], S.Y[p * LD + q]));
                        acc = c_add(acc, c_scale(w, z));
                    }
                    acc = c_scale(invN / de, c_i(acc));
                } else {
                    const double xm = 0.5 * (S.E[m] + S.E[q]);
                    double phx, dphx;
                    if (m == q) {
                        phx = S.phi[m];
                        dphx = S.dphi[m];
                    } else {
                        phi_at(xm, ef, sb, a.nF, a.kT, phx, dphx);
                    }
                    for (int p = 0; p < n; ++p) {
                        const double x = xm - S.E[p];
                        const double den = x * x + eta2;
                        const double w = dphx / den - (phx - S.phi[p]) * 2.0 * x / (den * den);
                        double2 z = c_mul(S.Y[m * LD + p], S.X[p * LD + q]);
                        z = c_sub(z, c_mul(S.X[m * LD + p], S.Y[p * LD + q]));
                        acc = c_add(acc, c_scale(w, z));
                    }
                    acc = c_scale(invN, c_i(acc));
                }
                S.A[m * LD + q] = acc;
            }
            __syncthreads();
            // Hbar = U Hbar' U^+  (T = Hbar' U^+, then A = U T)
            gemm_n_adjy<NT, LD>(S.T, S.A, S.V, n);
            __syncthreads();
            gemm_n<NT, LD, false>(S.A, S.V, S.T, n);
            __syncthreads();
            // vbar_x = U Abar U^+, Abar = (i/N) K o B  (T = Abar U^+, then Y = U T)
            for (int e = threadIdx.x; e < n * n; e += NT) {
                const int i = e / n, j = e - (e / n) * n;
                double2 acc = c_make(0.0, 0.0);
                for (int l = 0; l < n; ++l) {
                    const double2 ab = c_scale(invN * S.K[i * LD + l], c_i(S.Y[i * LD + l]));
                    acc = c_fma(ab, c_conj(S.V[j * LD + l]), acc);
                }
                S.T[i * LD + j] = acc;
            }
            __syncthreads();
            gemm_n<NT, LD, false>(S.Y, S.V, S.T, n);
            __syncthreads();
            // vbar_y = U Bbar U^+, Bbar = -(i/N) K o A  (T = Bbar U^+, then X = U T)
            for (int e = threadIdx.x; e < n * n; e += NT) {
                const int i = e / n, j = e - (e / n) * n;
                double2 acc = c_make(0.0, 0.0);
                for (int l = 0; l < n; ++l) {
                    const double2 bb = c_scale(-invN * S.K[i * LD + l], c_i(S.X[i * LD + l]));
                    acc = c_fma(bb, c_conj(S.V[j * LD + l]), acc);
                }
                S.T[i * LD + j] = acc;
            }
            __syncthreads();
            gemm_n<NT, LD, false>(S.X, S.V, S.T, n);
            __syncthreads();
            // pencil partials of the transposed Bloch sum
            for (long long e = threadIdx.x; e < (long long)md.nR0 * nn; e += NT) {
                const int rho = (int)(e / nn);
                const int ij = (int)(e - (long long)rho * nn);
                const int i = ij / n, j = ij - (ij / n) * n;
                const double2 pc = c_conj(S.ph[rho]);
                const double2 hb = S.A[i * LD + j];
                const double2 vx = S.Y[i * LD + j];
                const double2 vy = S.X[i * LD + j];
                // Hbar - i rho vbar_x
                const double2 w = c_sub(hb, c_scale((double)r0[rho], c_i(vx)));
                const double2 h1 = c_mul(pc, w);
                const double2 y1 = c_mul(pc, vy);
                if (!isfinite(h1.x + h1.y + y1.x + y1.y)) atomicOr(a.status, kStatNonFinite);
                if (kk == 0) {
                    PH[e] = h1;
                    PY[e] = y1;
                } else {
                    PH[e] = c_add(PH[e], h1);
                    PY[e] = c_add(PY[e], y1);
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// k_gacc: grad_t(R) += sum_{blocks} e^{-i(k1 R_y + k2 R_z)} (PH_rho - i R_y PY_rho), rho = R_x,
// for one range of k-blocks of one model (fixed order over the blocks).
// Grid: x = lattice vector in grouped order, y = tile of matrix entries, z = range.
// ---------------------------------------------------------------------------
constexpr int kGaccThreads = 256;
__global__ __launch_bounds__(kGaccThreads) void k_gacc(Tables tb, const GaccRange* __restrict__ ranges,
                                                       int range_begin,
                                                       const double2* __restrict__ pbuf,
                                                       double2* __restrict__ grad) {
    __shared__ double2 sph[kGaccThreads];
    __shared__ long long soff[kGaccThreads];
    const GaccRange rg = ranges[range_begin + blockIdx.z];
    const ModelDev md = tb.models[rg.model];
    const int g = blockIdx.x;
    if (g >= md.nR) return;
    const int n = md.n;
    const long long nn = (long long)n * n;
    const int gi = md.grp_first + g;
    const int r = tb.grp_r[gi];
    const int R1 = tb.grp_R1[gi], R2 = tb.grp_R2[gi];
    const int rho = tb.grp_rho[gi];
    const long long e = (long long)blockIdx.y * kGaccThreads + threadIdx.x;
    if ((long long)blockIdx.y * kGaccThreads >= nn) return;
    double2 acc = c_make(0.0, 0.0);
    for (int b0 = 0; b0 < rg.count; b0 += kGaccThreads) {
        const int bc = min(kGaccThreads, rg.count - b0);
        __syncthreads();
        if (threadIdx.x < bc) {
            const BlockItem bi = tb.blocks[rg.begin + b0 + threadIdx.x];
            sph[threadIdx.x] = unit_phase2(-(long long)bi.i1 * R1, md.N1, -(long long)bi.i2 * R2, md.N2);
            soff[threadIdx.x] = bi.pbuf_off;
        }
        __syncthreads();
        if (e < nn) {
            for (int b = 0; b < bc; ++b) {
                const double2* P = pbuf + soff[b];
                const double2 h = P[(long long)rho * nn + e];
                const double2 y = P[(long long)(md.nR0 + rho) * nn + e];
                const double2 w = c_sub(h, c_scale((double)R1, c_i(y)));
                acc = c_fma(sph[b], w, acc);
            }
        }
    }
    if (e < nn) {
        double2* G = grad + md.t_off + (long long)r * nn + e;
        *G = c_add(*G, acc);
    }
}

// grad_t(R) = (G'(R) + G'(-R)^+)/2: the chain rule through the Hermitian projection
// t'(R) = (t(R) + t(-R)^+)/2.  Each (R, -R) pair is handled by one thread, in place.
__global__ void k_gsym(Tables tb, int n_models, long long total, double2* __restrict__ grad) {
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; e < total; e += stride) {
        int lo = 0, hi = n_models - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (tb.models[mid].t_off <= e)
                lo = mid;
            else
                hi = mid - 1;
        }
        const ModelDev& md = tb.models[lo];
        const long long loc = e - md.t_off;
        const int n = md.n;
        const long long nn = (long long)n * n;
        const int r = (int)(loc / nn);
        const int ij = (int)(loc - (long long)r * nn);
        const int i = ij / n, j = ij - (ij / n) * n;
        const int rn = tb.negr[md.neg_first + r];
        const long long other = (long long)rn * nn + (long long)j * n + i;
        if (other < loc) continue;  // the partner thread owns the pair
        double2* pa = grad + md.t_off + loc;
        double2* pb = grad + md.t_off + other;
        const double2 a = *pa, b = *pb;
        const double2 v = c_make(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
        *pa = v;
        *pb = c_conj(v);
    }
}

// ---------------------------------------------------------------------------
// k_reduce: sigma[model][j] = -(1/N_k) sum_slots partial[slot][j], fixed order
// ---------------------------------------------------------------------------
constexpr int kReduceThreads = 256;
__global__ __launch_bounds__(kReduceThreads) void k_reduce(Tables tb, int nF,
                                                           const double* __restrict__ partial,
                                                           double* __restrict__ sigma,
                                                           unsigned* status) {
    __shared__ double red[kReduceThreads];
    const int m = blockIdx.y;
    const int j = blockIdx.x;
    const ModelDev md = tb.models[m];
    double s = 0.0;
    for (int k = threadIdx.x; k < md.slot_count; k += kReduceThreads)
        s += partial[(long long)(md.slot_first + k) * nF + j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double v = -red[0] / (double)md.Nk;
        if (!isfinite(v)) atomicOr(status, kStatNonFinite);
        sigma[md.f_off + j] = v;
    }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
hipError_t launch_clear(unsigned* status, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, status);
    return hipGetLastError();
}

hipError_t launch_zero(double* p, long long count, hipStream_t s) {
    long long blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_hermproj(const Tables& tb, int n_models, long long total, const double* t,
                           double* tp, hipStream_t s) {
    long long blocks = (total + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_hermproj, dim3((unsigned)blocks), dim3(256), 0, s, tb, n_models, total,
                       reinterpret_cast<const double2*>(t), reinterpret_cast<double2*>(tp));
    return hipGetLastError();
}

hipError_t launch_pencil(const Tables& tb, int item_begin, int item_count, const double* tp,
                         double* tbuf, hipStream_t s) {
    if (item_count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pencil, dim3(item_count), dim3(kPencilThreads), 0, s, tb, item_begin,
                       reinterpret_cast<const double2*>(tp), reinterpret_cast<double2*>(tbuf));
    return hipGetLastError();
}

template <int NP, int NT>
static hipError_t launch_forward_t(const FwdLaunch& L, hipStream_t s) {
    FwdArgs a;
    a.tb = L.tb;
    a.tbuf = reinterpret_cast<const double2*>(L.tbuf);
    a.e_fermi = L.e_fermi;
    a.partial = L.partial;
    a.status = L.status;
    a.eta = L.eta;
    a.kT = L.kT;
    a.nF = L.nF;
    a.max_sweeps = L.max_sweeps;
    a.item_begin = L.item_begin;
    a.item_count = L.item_count;
    const size_t lds = sizeof(FwdLds<NP, NT>);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_forward<NP, NT>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    int grid = L.item_count < L.max_groups ? L.item_count : L.max_groups;
    hipLaunchKernelGGL((k_forward<NP, NT>), dim3(grid), dim3(NT), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_forward(const FwdLaunch& L, hipStream_t s) {
    if (L.item_count <= 0) return hipSuccess;
    switch (L.np) {
        case 8:
            return launch_forward_t<8, 64>(L, s);
        case 16:
            return launch_forward_t<16, 128>(L, s);
        case 32:
            return launch_forward_t<32, 256>(L, s);
        default:
            return hipErrorInvalidValue;
    }
}

template <int NP, int NT>
static hipError_t launch_adjoint_t(const AdjLaunch& L, hipStream_t s) {
    AdjArgs a;
    a.tb = L.tb;
    a.tbuf = reinterpret_cast<const double2*>(L.tbuf);
    a.pbuf = reinterpret_cast<double2*>(L.pbuf);
    a.e_fermi = L.e_fermi;
    a.sbar = L.sbar;
    a.status = L.status;
    a.eta = L.eta;
    a.kT = L.kT;
    a.nF = L.nF;
    a.max_sweeps = L.max_sweeps;
    a.item_begin = L.item_begin;
    a.item_count = L.item_count;
    const size_t lds = sizeof(AdjLds<NP, NT>);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_adjoint<NP, NT>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    int grid = L.item_count < L.max_groups ? L.item_count : L.max_groups;
    hipLaunchKernelGGL((k_adjoint<NP, NT>), dim3(grid), dim3(NT), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_adjoint(const AdjLaunch& L, hipStream_t s) {
    if (L.item_count <= 0) return hipSuccess;
    switch (L.np) {
        case 8:
            return launch_adjoint_t<8, 64>(L, s);
        case 16:
            return launch_adjoint_t<16, 128>(L, s);
        case 32:
            return launch_adjoint_t<32, 256>(L, s);
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_gacc(const Tables& tb, const GaccRange* ranges, int range_begin, int range_count,
                       int max_nR, long long max_nn, const double* pbuf, double* grad,
                       hipStream_t s) {
    if (range_count <= 0) return hipSuccess;
    const unsigned ty = (unsigned)((max_nn + kGaccThreads - 1) / kGaccThreads);
    hipLaunchKernelGGL(k_gacc, dim3(max_nR, ty, range_count), dim3(kGaccThreads), 0, s, tb,
                       ranges, range_begin, reinterpret_cast<const double2*>(pbuf),
                       reinterpret_cast<double2*>(grad));
    return hipGetLastError();
}

hipError_t launch_gsym(const Tables& tb, int n_models, long long total, double* grad,
                       hipStream_t s) {
    long long blocks = (total + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_gsym, dim3((unsigned)blocks), dim3(256), 0, s, tb, n_models, total,
                       reinterpret_cast<double2*>(grad));
    return hipGetLastError();
}

hipError_t launch_reduce(const Tables& tb, int n_models, int nF, const double* partial,
                         double* sigma, unsigned* status, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(nF, n_models), dim3(kReduceThreads), 0, s, tb, nF, partial,
                       sigma, status);
    return hipGetLastError();
}

}  // namespace kubo
