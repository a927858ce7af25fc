// kubo_gf.hip -- the Green's-function form of sigma_xy (n <= 32).
//
// The paper remarks, after Eq. (3), that systems with impurities need Green's
// functions -- matrix inverses -- instead of eigenvalues.  With a constant
// scattering rate gamma, G = ((i (w + gamma) + mu) I - H(k))^{-1} and
//   sigma(mu) = (1/N_k) sum_k int_0^inf dw/(2 pi) Im{Tr[G v_x G G v_y] - Tr[G v_y G G v_x]},
// the w-integral given as caller nodes and weights.  At gamma = 0 this equals
// Eqs. (2)-(3) at zero temperature (the poles at w = i (mu - E_n) give the
// band-pair sum), so it reuses the pencil partial sums of step 1 and replaces
// the eigensolve of step 2 and the rotations of step 3 by one inverse and four
// products per Fermi level and node.
//
// k_gf: one 256-thread workgroup per k-point.  H lives in registers (thread t
// owns row t / 8, columns t % 8 + 8 q), v_x and v_y too, as the MFMA B operands of
// the lane's quadrant column; G and the two products X = G v_x, Y = G v_y live in
// LDS (32 x 33 complex each, 51 KB: three workgroups per CU).  The
// inverse is Gauss-Jordan elimination without pivoting: (i (w + gamma) + mu) - H
// times -i has the positive definite Hermitian part (w + gamma) I, so every
// pivot is nonzero and elimination without pivoting is stable for it.  The four
// products (X, Y, X G and Y G) run on FP64 MFMA, each wavefront one 16 x 16
// quadrant; Tr[X G Y] and Tr[Y G X] are taken from the product accumulators
// against the transposed third factor in LDS, so X G and Y G are never stored.
#include <hip/hip_runtime.h>

#include <cstddef>

#include "kubo_cplx.h"
#include "kubo_internal.h"
#include "kubo_launch.h"

namespace kubo {

namespace {

constexpr int kGfN = 32;
constexpr int kGfLD = kGfN + 1;
constexpr int kGfThreads = 256;

struct GfLds {
    double2 G[kGfN * kGfLD];
    double2 X[kGfN * kGfLD];
    double2 Y[kGfN * kGfLD];
    double2 row[2][kGfN];  // pivot row of the elimination, by step parity
    double2 col[2][kGfN];  // pivot column
    double2 ph[16];        // e^{i k0 rho} of the k-point
    double red[kGfThreads / 64];
};

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// C (16 x 16 quadrant at rows r0, columns c0) += A B over the inner index
// k < kmax (kmax a multiple of 4, <= 32); A and B row-major in LDS.  Lane l
// supplies A[r0 + l % 16][k0 + l / 16] and B[k0 + l / 16][c0 + l % 16] and ends
// with C[r0 + l / 16 + 4 q][c0 + l % 16] in element q of (cr, ci).
__device__ __forceinline__ void gf_mm(const double2* A, const double2* B, int r0, int c0, int kmax,
                                      int lane, v4d& cr, v4d& ci) {
    const int a_row = r0 + (lane & 15), b_col = c0 + (lane & 15), kl = lane >> 4;
    for (int k0 = 0; k0 < kmax; k0 += 4) {
        const double2 a = A[a_row * kGfLD + k0 + kl];
        const double2 b = B[(k0 + kl) * kGfLD + b_col];
        cr = mfma(a.x, b.x, cr);
        cr = mfma(-a.y, b.y, cr);
        ci = mfma(a.x, b.y, ci);
        ci = mfma(a.y, b.x, ci);
    }
}

// The same with B given as this lane's operands b[k0 / 4] = B[k0 + lane / 16][c0 + lane % 16].
__device__ __forceinline__ void gf_mm_rb(const double2* A, const double2 (&b)[kGfN / 4], int r0,
                                         int kmax, int lane, v4d& cr, v4d& ci) {
    const int a_row = r0 + (lane & 15), kl = lane >> 4;
#pragma unroll
    for (int s = 0; s < kGfN / 4; ++s) {
        if (4 * s < kmax) {
            const double2 a = A[a_row * kGfLD + 4 * s + kl];
            cr = mfma(a.x, b[s].x, cr);
            cr = mfma(-a.y, b[s].y, cr);
            ci = mfma(a.x, b[s].y, ci);
            ci = mfma(a.y, b[s].x, ci);
        }
    }
}

__device__ __forceinline__ double gf_wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// 1 / z: the hardware reciprocal estimate of |z|^2 and one Newton step
__device__ __forceinline__ double2 c_recip(double2 z) {
    const double m = fma(z.x, z.x, z.y * z.y);
    double d = __builtin_amdgcn_rcp(m);
    d = fma(d, fma(-m, d, 1.0), d);
    return c_make(z.x * d, -z.y * d);
}

}  // namespace

__global__ __launch_bounds__(kGfThreads, 3) void k_gf(GfLaunch a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    GfLds& S = *reinterpret_cast<GfLds*>(smem_raw);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int ri = tid >> 3, cj0 = tid & 7;  // owned elements (ri, cj0 + 8 q)
    const int qr0 = (wave >> 1) * 16, qc0 = (wave & 1) * 16;  // this wavefront's quadrant
    const double2* tbuf = reinterpret_cast<const double2*>(a.tbuf);
    const double inv2pi = 0.15915494309189533577;
    int probe = 0;
    for (int par = 0;; par ^= 1) {
        __shared__ int unit[2];
        if (tid == 0) unit[par] = queue_take(a.queue, a.item_count, probe);
        __syncthreads();
        const int item = unit[par];
        if (item < 0) break;
        const BlockItem it = a.tb.blocks[a.item_begin + item];
        const ModelDev md = a.tb.models[it.model];
        const int n = md.n;
        const long long nn = (long long)n * n;
        const double2* T0 = tbuf + it.tbuf_off;
        const double2* T1 = T0 + (long long)md.nR0 * nn;
        const int* r0 = a.tb.r0val + md.r0_first;
        const double* ef = a.e_fermi + md.f_off;
        double* part = a.partial + (long long)it.slot * a.nF;
        const int kq = (n + 3) & ~3;  // inner extent of the products
        const bool quad_live = qr0 < n && qc0 < n;
        for (int kk = 0; kk < it.count; ++kk) {
            // ---- step 1: H, v_x and v_y (registers) from the pencil partial sums
            if (tid < md.nR0) S.ph[tid] = unit_phase((long long)(it.i0 + kk) * r0[tid], md.N0);
            __syncthreads();
            double2 h[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = cj0 + 8 * q;
                double2 hv = c_make(0.0, 0.0), xv = c_make(0.0, 0.0), yv = c_make(0.0, 0.0);
                if (ri < n && j < n) {
                    for (int rho = 0; rho < md.nR0; ++rho) {
                        const double2 ph = S.ph[rho];
                        const double2 t0 = T0[rho * nn + ri * n + j];
                        const double2 t1 = T1[rho * nn + ri * n + j];
                        hv = c_fma(t0, ph, hv);
                        xv = c_fma(t0, c_scale((double)r0[rho], c_i(ph)), xv);
                        yv = c_fma(t1, ph, yv);
                    }
                }
                h[q] = hv;
                S.X[ri * kGfLD + j] = xv;  // v_x and v_y pass through the X and Y buffers
                S.Y[ri * kGfLD + j] = yv;
            }
            __syncthreads();
            double2 bx[kGfN / 4], by[kGfN / 4];
#pragma unroll
            for (int s4 = 0; s4 < kGfN / 4; ++s4) {
                const int e = (4 * s4 + (lane >> 4)) * kGfLD + qc0 + (lane & 15);
                bx[s4] = S.X[e];
                by[s4] = S.Y[e];
            }
            __syncthreads();
            for (int fj = 0; fj < a.nF; ++fj) {
                double acc = 0.0;  // thread 0: sum over the nodes
                for (int l = 0; l < a.n_omega; ++l) {
                    // ---- A = (i (w + gamma) + mu) I - H; identity on the padding
                    const double2 z = c_make(ef[fj], a.omega[l] + a.gamma);
                    double2 g[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int j = cj0 + 8 * q;
                        if (ri < n && j < n)
                            g[q] = (ri == j) ? c_sub(z, h[q]) : c_make(-h[q].x, -h[q].y);
                        else
                            g[q] = c_make(ri == j ? 1.0 : 0.0, 0.0);
                    }
                    // ---- Gauss-Jordan inverse in place, one barrier per step
                    for (int p = 0; p < n; ++p) {
                        const int b = p & 1;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int j = cj0 + 8 * q;
                            if (ri == p) S.row[b][j] = g[q];
                            if (j == p) S.col[b][ri] = g[q];
                        }
                        __syncthreads();
                        const double2 piv = c_recip(S.row[b][p]);
                        const double2 cp = S.col[b][ri];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int j = cj0 + 8 * q;
                            const double2 rs = c_mul(S.row[b][j], piv);
                            if (ri == p)
                                g[q] = (j == p) ? piv : rs;
                            else if (j == p)
                                g[q] = c_make(-(cp.x * piv.x - cp.y * piv.y), -(cp.x * piv.y + cp.y * piv.x));
                            else
                                g[q] = c_fnma(cp, rs, g[q]);
                        }
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) S.G[ri * kGfLD + cj0 + 8 * q] = g[q];
                    __syncthreads();
                    // ---- X = G v_x, Y = G v_y
                    {
                        v4d xr = {0.0, 0.0, 0.0, 0.0}, xi = xr, yr = xr, yi = xr;
                        if (quad_live) {
                            gf_mm_rb(S.G, bx, qr0, kq, lane, xr, xi);
                            gf_mm_rb(S.G, by, qr0, kq, lane, yr, yi);
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int e = (qr0 + (lane >> 4) + 4 * q) * kGfLD + qc0 + (lane & 15);
                            S.X[e] = c_make(xr[q], xi[q]);
                            S.Y[e] = c_make(yr[q], yi[q]);
                        }
                    }
                    __syncthreads();
                    // ---- Im Tr[X G Y] - Im Tr[Y G X] from the quadrants of X G and Y G
                    double im = 0.0;
                    if (quad_live) {
                        v4d cr = {0.0, 0.0, 0.0, 0.0}, ci = cr, dr = cr, di = cr;
                        gf_mm(S.X, S.G, qr0, qc0, kq, lane, cr, ci);
                        gf_mm(S.Y, S.G, qr0, qc0, kq, lane, dr, di);
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int r = qr0 + (lane >> 4) + 4 * q, c = qc0 + (lane & 15);
                            const double2 yt = S.Y[c * kGfLD + r], xt = S.X[c * kGfLD + r];
                            im += cr[q] * yt.y + ci[q] * yt.x;  // Im((X G)_rc Y_cr)
                            im -= dr[q] * xt.y + di[q] * xt.x;  // Im((Y G)_rc X_cr)
                        }
                    }
                    im = gf_wave_sum(im);
                    if (lane == 0) S.red[wave] = im;
                    __syncthreads();
                    if (tid == 0) {
                        const double v = (S.red[0] + S.red[1]) + (S.red[2] + S.red[3]);
                        acc = fma(a.weight[l] * inv2pi, v, acc);
                    }
                }
                if (tid == 0) {
                    // sigma = -(1/N_k) sum of the partials
                    const double v = -acc;
                    if (!isfinite(v)) atomicOr(a.status, kStatNonFinite);
                    part[fj] = (kk == 0) ? v : part[fj] + v;
                }
            }
            __syncthreads();
        }
    }
}

hipError_t launch_gf(const GfLaunch& L, hipStream_t s) {
    if (L.item_count <= 0) return hipSuccess;
    if (!L.queue || L.n_omega < 1) return hipErrorInvalidValue;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gf),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)sizeof(GfLds));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int grid = L.item_count < L.max_groups ? L.item_count : L.max_groups;
    hipLaunchKernelGGL(k_gf, dim3(grid), dim3(kGfThreads), sizeof(GfLds), s, L);
    return hipGetLastError();
}

}  // namespace kubo
