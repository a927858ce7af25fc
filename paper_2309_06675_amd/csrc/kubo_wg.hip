// kubo_wg.hip -- one workgroup (256 threads) per k-point for 32 < n <= 128,
// forward and adjoint.
//
// Same method as the one-wavefront path (Householder reduction to a real
// tridiagonal matrix, Sturm counts with safeguarded Newton steps for the
// eigenvalues, twisted factorisations for the eigenvectors with an implicit-QL
// path for clustered spectra, back-transformation, U^+ v U), but the n x n
// matrices of the k-point being processed live in a per-workgroup slice of the
// workspace (it stays in L2 / the last-level cache) instead of registers and
// LDS, which cannot hold them all at n = 128.  Two instantiations: n <= 64
// (reduction on an LDS copy of the matrix, products on the FP64 matrix cores,
// two workgroups per CU) and n <= 128 (reduction on the lower triangle packed
// into LDS, products through 32 x 32 LDS tiles, one workgroup per CU with the
// CU's whole LDS); both keep the twisted factorisations' pivots in LDS and U in
// registers for the back-transformation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>

#include "kubo_cplx.h"
#include "kubo_internal.h"
#include "kubo_launch.h"

namespace kubo {

constexpr int kWgThreads = 256;
// Eigenvalues closer than this fraction of the spectral span send the k-point to the
// implicit-QL path; wider gaps take one twisted factorisation per eigenvector, whose
// error (like that of any backward-stable eigensolver) is of order eps |T| / gap.
constexpr double kWgClusterGap = 1e-5;
constexpr int kWgMaxN = 128;
constexpr int kTile = 32;

struct WgLds {
    // used by the Householder reduction
    double2 xv[kWgMaxN];
    double2 vv[kWgMaxN];
    double2 wv[kWgMaxN];
    double2 tau[kWgMaxN];
    double d[kWgMaxN];
    double e[kWgMaxN];
    double2 ph[16];
    double red[2 * (kWgThreads / 64)];
    int flag;
    int unit[2];  // work unit taken by thread 0, double-buffered by loop parity
    // dead during the reduction from lam on: the n <= 64 kernels put the
    // matrix there (over the end of the struct, into their dynamic extension);
    // 16-byte aligned so that its complex elements are aligned
    alignas(16) double lam[kWgMaxN];
    double cs[2 * kWgMaxN];
    double en[kWgMaxN];
    double dn[kWgMaxN];
    double E[kWgMaxN];
    double Om[kWgMaxN];
    double phi[kWgMaxN];
    double dphi[kWgMaxN];
    // Hall tensor: curvatures of the (v_y, v_z), (v_z, v_x), (Js_x, v_y) pairs
    double Om2[3][kWgMaxN];
    // From here to the end of the dynamic allocation: one scratch region shared by
    // phases that never overlap (GEMM tiles, staged reflectors, twisted pivots)
    double2 ta[kTile * (kTile + 1)];
    double2 tb[kTile * (kTile + 1)];
};

// The n <= 64 kernels get 80 KB of LDS per workgroup (two workgroups per CU):
// the n x n matrix of the Householder reduction from S.lam on, and the four
// wavefronts' partial sums of p (4 x 64 complex) at the very end.
constexpr size_t kWgSmallLds = 80 * 1024;
// The n <= 128 kernels (one workgroup per CU) take the whole LDS of the CU.
constexpr size_t kWgBigLds = 160 * 1024;
constexpr int kWgSmallN = 64;
constexpr size_t kWgSmallPart = sizeof(double2) * (kWgThreads / 64) * kWgSmallN;
static_assert(sizeof(WgLds) <= kWgSmallLds, "LDS layout");
static_assert(offsetof(WgLds, lam) % 16 == 0 && offsetof(WgLds, ta) % 16 == 0, "LDS alignment");
static_assert(offsetof(WgLds, ta) + sizeof(double2) * kWgMaxN * (kWgMaxN + 1) / 2 <= kWgBigLds,
              "packed matrix in the LDS scratch region");
// the scratch region: from ta to the end of the dynamic allocation
__device__ __forceinline__ double* wg_region(WgLds& S) { return reinterpret_cast<double*>(S.ta); }
template <bool SMALL>
__host__ __device__ constexpr size_t wg_region_doubles() {
    return ((SMALL ? kWgSmallLds : kWgBigLds) - offsetof(WgLds, ta)) / sizeof(double);
}
static_assert(offsetof(WgLds, lam) + sizeof(double2) * kWgSmallN * kWgSmallN <= kWgSmallLds - kWgSmallPart,
              "LDS matrix region");

// Per-workgroup scratch: seven n_max x n_max complex matrices.
struct WgScratch {
    double2* P;    // H, then Householder vectors; adjoint: product scratch
    double2* U;    // Z, then U
    double2* VX;   // v_x, then A = U^+ v_x U; adjoint: vbar_y
    double2* VY;   // v_y, then B = U^+ v_y U; adjoint: vbar_x
    double2* W;    // product scratch; adjoint: Hbar', then Hbar
    double* DPM;   // pivots of the twisted factorisations (2 n^2 doubles)
    double* K;     // adjoint: K_mn (n^2 doubles)
};

__device__ __forceinline__ WgScratch wg_scratch(double2* base, long long slot_elems, int slot) {
    const long long m2 = slot_elems / 7;
    double2* b = base + (long long)slot * slot_elems;
    WgScratch s;
    s.P = b;
    s.U = b + m2;
    s.VX = b + 2 * m2;
    s.VY = b + 3 * m2;
    s.W = b + 4 * m2;
    s.DPM = reinterpret_cast<double*>(b + 5 * m2);
    s.K = reinterpret_cast<double*>(b + 6 * m2);
    return s;
}

// Wavefront reduction without the LDS crossbar: DPP within rows of 16 lanes,
// then the gfx950 row swaps (v_permlane16_swap, v_permlane32_swap); every lane
// ends with the same bits.
template <class Op>
__device__ __forceinline__ double wg_wave_reduce(double v, Op op) {
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));   // lane ^ 1
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));   // lane ^ 2
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false));  // 7 - lane within 8
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false));  // 15 - lane within 16
    auto join = [](unsigned lo, unsigned hi) {
        return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
    };
    {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
        v = op(join(lo[0], hi[0]), join(lo[1], hi[1]));
    }
    {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
        v = op(join(lo[0], hi[0]), join(lo[1], hi[1]));
    }
    return v;
}

// value of a per-lane register held by lane src of the wavefront (src wave-uniform)
__device__ __forceinline__ double wg_lane_read(double v, int src) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), src);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Workgroup sum of one double (all threads get the result).
__device__ __forceinline__ double wg_sum(double v, double* red) {
    v = wg_wave_reduce(v, [](double x, double y) { return x + y; });
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kWgThreads / 64; ++w) s += red[w];
    __syncthreads();
    return s;
}
__device__ __forceinline__ double wg_min(double v, double* red) {
    v = wg_wave_reduce(v, [](double x, double y) { return fmin(x, y); });
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
    for (int w = 1; w < kWgThreads / 64; ++w) s = fmin(s, red[w]);
    __syncthreads();
    return s;
}
__device__ __forceinline__ double wg_max(double v, double* red) {
    return -wg_min(-v, red);
}

// ---------------------------------------------------------------------------
// step 1: H (Hermitian, upper triangle mirrored), v_x, v_y into the scratch
// ---------------------------------------------------------------------------
__device__ void wg_build(WgLds& S, const WgScratch& X, const ModelDev& md,
                         const double2* __restrict__ T0, const double2* __restrict__ T1,
                         const int* __restrict__ r0, int i0) {
    const int n = md.n;
    const long long nn = (long long)n * n;
    if (threadIdx.x < md.nR0) S.ph[threadIdx.x] = unit_phase((long long)i0 * r0[threadIdx.x], md.N0);
    __syncthreads();
    // H, v_x and v_y are Hermitian (the hoppings are Hermitian-projected): the
    // upper triangles are summed, packed row by row, and mirrored
    const int nu = n * (n + 1) / 2;
    for (int e = threadIdx.x; e < nu; e += kWgThreads) {
        // row i starts at s(i) = i n - i (i - 1) / 2
        const float b = 2.0f * n + 1.0f;
        int i = (int)(0.5f * (b - sqrtf(b * b - 8.0f * (float)e)));
        if (i * n - (i * (i - 1)) / 2 > e) --i;
        else if ((i + 1) * n - ((i + 1) * i) / 2 <= e) ++i;
        const int j = i + (e - (i * n - (i * (i - 1)) / 2));
        const long long off = (long long)i * n + j;
        double2 h = c_make(0.0, 0.0), x = h, y = h;
        // four rho terms' loads issued together (the index clamped, so every load is
        // valid), then their sums
        for (int r4 = 0; r4 < md.nR0; r4 += 4) {
            double2 t0[4], t1[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const long long o = (long long)min(r4 + u, md.nR0 - 1) * nn + off;
                t0[u] = T0[o];
                t1[u] = T1[o];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int rho = r4 + u;
                if (rho < md.nR0) {
                    const double2 p0 = c_mul(t0[u], S.ph[rho]);
                    h = c_add(h, p0);
                    x = c_add(x, c_scale((double)r0[rho], c_i(p0)));
                    y = c_fma(t1[u], S.ph[rho], y);
                }
            }
        }
        if (i == j) {
            h.y = 0.0;
            x.y = 0.0;
            y.y = 0.0;
        }
        X.P[i * n + j] = h;
        X.P[j * n + i] = c_conj(h);
        X.VX[i * n + j] = x;
        X.VX[j * n + i] = c_conj(x);
        X.VY[i * n + j] = y;
        X.VY[j * n + i] = c_conj(y);
    }
    __syncthreads();
}

// Hall tensor: v_z (from the third set of pencil partials) into VZ and, when spin is
// given, the spin current Js_x = (s v_x + v_x s)/2 into JS (n x n each, Hermitian,
// upper triangles summed and mirrored).
__device__ void wg_build_tensor(WgLds& S, const ModelDev& md, const double2* __restrict__ T0,
                                const double2* __restrict__ T2, const int* __restrict__ r0, int i0,
                                const double* __restrict__ spin, double2* __restrict__ VZ,
                                double2* __restrict__ JS) {
    const int n = md.n;
    const long long nn = (long long)n * n;
    if (threadIdx.x < md.nR0) S.ph[threadIdx.x] = unit_phase((long long)i0 * r0[threadIdx.x], md.N0);
    __syncthreads();
    const int nu = n * (n + 1) / 2;
    for (int e = threadIdx.x; e < nu; e += kWgThreads) {
        const float b = 2.0f * n + 1.0f;
        int i = (int)(0.5f * (b - sqrtf(b * b - 8.0f * (float)e)));
        if (i * n - (i * (i - 1)) / 2 > e) --i;
        else if ((i + 1) * n - ((i + 1) * i) / 2 <= e) ++i;
        const int j = i + (e - (i * n - (i * (i - 1)) / 2));
        const long long off = (long long)i * n + j;
        double2 z = c_make(0.0, 0.0), x = z;
        for (int rho = 0; rho < md.nR0; ++rho) {
            z = c_fma(T2[(long long)rho * nn + off], S.ph[rho], z);
            if (spin) x = c_add(x, c_scale((double)r0[rho], c_i(c_mul(T0[(long long)rho * nn + off], S.ph[rho]))));
        }
        if (i == j) {
            z.y = 0.0;
            x.y = 0.0;
        }
        VZ[i * n + j] = z;
        VZ[j * n + i] = c_conj(z);
        if (spin) {
            x = c_scale(0.5 * (spin[i] + spin[j]), x);
            JS[i * n + j] = x;
            JS[j * n + i] = c_conj(x);
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// step 2a for n <= 128 on the lower triangle of the matrix packed into LDS
// (element (r, c), c <= r, at r (r + 1) / 2 + c; 132 KB at n = 128), the same
// steps as wg_tridiag: column k through LDS, its reflector, p = A22 v (two
// threads per row, the upper triangle read as the conjugate of the lower one),
// w, and the rank-2 update of the trailing lower triangle (two threads per
// column, lanes over columns so that a row's elements are consecutive).  The
// reflectors are written back into P (column k below the diagonal) for the
// back-transformation.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int tri_idx(int r, int c) { return (r * (r + 1)) / 2 + c; }

__device__ void wg_tridiag_packed(WgLds& S, double2* __restrict__ P, int n, double2* __restrict__ L) {
    const int tid = threadIdx.x;
    const int nt = n * (n + 1) / 2;
    // row of packed element e: the largest r with r (r + 1) / 2 <= e (float estimate, corrected)
    auto tri_row = [](int e) {
        int r = (int)(0.5f * (sqrtf(8.0f * (float)e + 1.0f) - 1.0f));
        if (tri_idx(r, 0) > e) --r;
        else if (tri_idx(r + 1, 0) <= e) ++r;
        return r;
    };
    for (int e = tid; e < nt; e += kWgThreads) {
        const int r = tri_row(e);
        L[e] = P[r * n + (e - tri_idx(r, 0))];
    }
    __syncthreads();
    auto rcp = [](double x) {
        const double r0 = __builtin_amdgcn_rcp(x);
        return fma(r0, fma(-x, r0, 1.0), r0);
    };
    for (int k = 0; k < n - 1; ++k) {
        double part = 0.0;
        for (int r = k + 1 + tid; r < n; r += kWgThreads) {
            const double2 x = L[tri_idx(r, k)];
            S.xv[r] = x;
            if (r > k + 1) part = fma(x.x, x.x, fma(x.y, x.y, part));
        }
        const double xn2 = wg_sum(part, S.red);
        const double2 alpha = S.xv[k + 1];
        double beta;
        double2 tau, scal;
        if (xn2 == 0.0 && alpha.y == 0.0) {
            beta = alpha.x;
            tau = c_make(0.0, 0.0);
            scal = c_make(0.0, 0.0);
        } else {
            const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2);
            beta = -copysign(nrm, alpha.x);
            const double ib = rcp(beta);
            tau = c_make((beta - alpha.x) * ib, -alpha.y * ib);
            const double ar = alpha.x - beta, ai = alpha.y;
            const double den = rcp(ar * ar + ai * ai);
            scal = c_make(ar * den, -ai * den);
        }
        if (tid == 0) {
            S.d[k] = L[tri_idx(k, k)].x;
            S.e[k] = beta;
            S.tau[k] = tau;
        }
        for (int r = k + 1 + tid; r < n; r += kWgThreads) {
            const double2 v = (r == k + 1) ? c_make(1.0, 0.0) : c_mul(S.xv[r], scal);
            S.vv[r] = v;
            L[tri_idx(r, k)] = v;
        }
        __syncthreads();
        if (tau.x == 0.0 && tau.y == 0.0) continue;
        // p = A22 v: rows over thread pairs, the pair's two threads over alternate
        // columns; the row part (c <= r, consecutive words) and the column part (c > r,
        // the conjugate of row c) as separate loops, four independent sums each
        for (int r = k + 1 + (tid >> 1); r < n; r += kWgThreads / 2) {
            double2 p0 = c_make(0.0, 0.0), p1 = p0, p2 = p0, p3 = p0;
            const int rb = tri_idx(r, 0);
            int c = k + 1 + (tid & 1);
            for (; c + 6 <= r; c += 8) {
                p0 = c_fma(L[rb + c], S.vv[c], p0);
                p1 = c_fma(L[rb + c + 2], S.vv[c + 2], p1);
                p2 = c_fma(L[rb + c + 4], S.vv[c + 4], p2);
                p3 = c_fma(L[rb + c + 6], S.vv[c + 6], p3);
            }
            for (; c <= r; c += 2) p0 = c_fma(L[rb + c], S.vv[c], p0);
            for (; c + 6 < n; c += 8) {
                p0 = c_fmac(L[tri_idx(c, r)], S.vv[c], p0);
                p1 = c_fmac(L[tri_idx(c + 2, r)], S.vv[c + 2], p1);
                p2 = c_fmac(L[tri_idx(c + 4, r)], S.vv[c + 4], p2);
                p3 = c_fmac(L[tri_idx(c + 6, r)], S.vv[c + 6], p3);
            }
            for (; c < n; c += 2) p0 = c_fmac(L[tri_idx(c, r)], S.vv[c], p0);
            double2 p = c_add(c_add(p0, p1), c_add(p2, p3));
            p.x += __shfl_xor(p.x, 1, 64);
            p.y += __shfl_xor(p.y, 1, 64);
            if ((tid & 1) == 0) S.wv[r] = p;
        }
        __syncthreads();
        double mpart = 0.0;
        for (int r = k + 1 + tid; r < n; r += kWgThreads) mpart += S.vv[r].x * S.wv[r].x + S.vv[r].y * S.wv[r].y;
        const double mu = wg_sum(mpart, S.red);
        const double t2 = 0.5 * (tau.x * tau.x + tau.y * tau.y) * mu;
        for (int r = k + 1 + tid; r < n; r += kWgThreads)
            S.wv[r] = c_sub(c_mul(tau, S.wv[r]), c_scale(t2, S.vv[r]));
        __syncthreads();
        // trailing lower triangle: lanes over the columns c (a row's elements are
        // consecutive), the two halves of the workgroup over alternate rows r >= c
        {
            const int c = k + 1 + (tid & 127), h = tid >> 7;
            const double2 vc = (c < n) ? S.vv[c] : c_make(0.0, 0.0);
            const double2 wc = (c < n) ? S.wv[c] : c_make(0.0, 0.0);
            int r = k + 1 + h;
            for (; r + 6 < n; r += 8) {
                double2 x[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (c <= r + 2 * u) x[u] = L[tri_idx(r + 2 * u, c)];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (c <= r + 2 * u)
                        L[tri_idx(r + 2 * u, c)] = c_rank2c(x[u], S.vv[r + 2 * u], wc, S.wv[r + 2 * u], vc);
            }
            for (; r < n; r += 2) {
                if (c <= r) {
                    const int ix = tri_idx(r, c);
                    L[ix] = c_rank2c(L[ix], S.vv[r], wc, S.wv[r], vc);
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        S.d[n - 1] = L[tri_idx(n - 1, n - 1)].x;
        S.e[n - 1] = 0.0;
    }
    // the reflectors back to P, column k below the diagonal
    for (int e = tid; e < nt; e += kWgThreads) {
        const int r = tri_row(e);
        const int c = e - tri_idx(r, 0);
        if (c < r) P[r * n + c] = L[e];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// step 2a for n <= 64, the same reduction on an LDS copy of the whole matrix.
// Per step: the reflector from column k (held in S.xv with its norm partials);
// p = A22 v in column form (A22 is Hermitian, p_r = sum_c conj(A_cr) v_c), each
// wavefront summing every fourth c with lanes over r into an LDS buffer (part),
// together with its share of v^+ p; the rank-2 update with wavefronts over rows
// and lanes over columns, w formed where it is needed from the partial sums of
// p, and the lane holding column k + 1 keeping that column and its norm
// partials for the next step.  Three barriers per step.
// ---------------------------------------------------------------------------
__device__ void wg_tridiag_cols(WgLds& S, double2* __restrict__ P, int n, double2* __restrict__ part) {
    // part: [NW][kWgSmallN] partial sums of p (n <= kWgSmallN)
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    constexpr int NW = kWgThreads / 64;
    auto rcp = [](double x) {
        const double r = __builtin_amdgcn_rcp(x);
        return fma(r, fma(-x, r, 1.0), r);
    };
    auto wave_sum = [](double v) { return wg_wave_reduce(v, [](double x, double y) { return x + y; }); };
    // column 0 and the partial sums of its squared norm below the subdiagonal (S.red[0..NW))
    {
        double nrm_part = 0.0;
        for (int r = 1 + tid; r < n; r += kWgThreads) {
            const double2 x = P[r * n];
            S.xv[r] = x;
            if (r > 1) nrm_part = fma(x.x, x.x, fma(x.y, x.y, nrm_part));
        }
        nrm_part = wave_sum(nrm_part);
        if (lane == 0) S.red[w] = nrm_part;
        __syncthreads();
    }
    for (int k = 0; k < n - 1; ++k) {
        // S.xv holds column k (rows > k), S.red[0..NW) its norm partials
        const double xn2 = (S.red[0] + S.red[1]) + (S.red[2] + S.red[3]);
        const double2 alpha = S.xv[k + 1];
        double beta;
        double2 tau, scal;
        if (xn2 == 0.0 && alpha.y == 0.0) {
            beta = alpha.x;
            tau = c_make(0.0, 0.0);
            scal = c_make(0.0, 0.0);
        } else {
            const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2);
            beta = -copysign(nrm, alpha.x);
            const double ib = rcp(beta);
            tau = c_make((beta - alpha.x) * ib, -alpha.y * ib);
            const double ar = alpha.x - beta, ai = alpha.y;
            const double den = rcp(ar * ar + ai * ai);
            scal = c_make(ar * den, -ai * den);
        }
        if (tid == 0) {
            S.d[k] = P[k * n + k].x;
            S.e[k] = beta;
            S.tau[k] = tau;
        }
        for (int r = k + 1 + tid; r < n; r += kWgThreads) {
            const double2 v = (r == k + 1) ? c_make(1.0, 0.0) : c_mul(S.xv[r], scal);
            S.vv[r] = v;
            P[r * n + k] = v;
        }
        __syncthreads();
        if (tau.x == 0.0 && tau.y == 0.0) {
            // nothing to reflect: the next column as it stands
            double nrm_part = 0.0;
            for (int r = k + 2 + tid; r < n; r += kWgThreads) {
                const double2 x = P[r * n + k + 1];
                S.xv[r] = x;
                if (r > k + 2) nrm_part = fma(x.x, x.x, fma(x.y, x.y, nrm_part));
            }
            nrm_part = wave_sum(nrm_part);
            __syncthreads();
            if (lane == 0) S.red[w] = nrm_part;
            __syncthreads();
            continue;
        }
        // partial p_r over c = k + 1 + w (mod NW), two interleaved accumulators, and this
        // wavefront's share of mu = v^+ p (real) into S.red[NW + w]
        double mpart = 0.0;
        for (int r = k + 1 + lane; r < n; r += 64) {
            double2 a0 = c_make(0.0, 0.0), a1 = a0;
            int c = k + 1 + w;
            for (; c + NW < n; c += 2 * NW) {
                a0 = c_fmac(P[c * n + r], S.vv[c], a0);
                a1 = c_fmac(P[(c + NW) * n + r], S.vv[c + NW], a1);
            }
            if (c < n) a0 = c_fmac(P[c * n + r], S.vv[c], a0);
            const double2 pw = c_add(a0, a1);
            part[w * kWgSmallN + r] = pw;
            const double2 vr = S.vv[r];
            mpart = fma(vr.x, pw.x, fma(vr.y, pw.y, mpart));
        }
        mpart = wave_sum(mpart);
        if (lane == 0) S.red[NW + w] = mpart;
        __syncthreads();
        const double mu = (S.red[NW] + S.red[NW + 1]) + (S.red[NW + 2] + S.red[NW + 3]);
        const double t2 = 0.5 * (tau.x * tau.x + tau.y * tau.y) * mu;
        // w_r = tau p_r - t2 v_r, formed where it is needed from the four partial sums of p
        auto w_of = [&](int r) {
            const double2 pr = c_add(c_add(part[r], part[kWgSmallN + r]),
                                     c_add(part[2 * kWgSmallN + r], part[3 * kWgSmallN + r]));
            return c_sub(c_mul(tau, pr), c_scale(t2, S.vv[r]));
        };
        // A22 <- A22 - v w^+ - w v^+: wavefronts over rows, lanes over columns; the lane
        // holding column k + 1 keeps the updated column for the next step and the partial
        // sums of its squared norm below the next subdiagonal
        const int c = k + 1 + lane;  // n <= 64: one column per lane
        const double2 wc = (c < n) ? w_of(c) : c_make(0.0, 0.0);
        const double2 vc = (c < n) ? S.vv[c] : c_make(0.0, 0.0);
        double nrm_part = 0.0;
        for (int rr = k + 1 + w; rr < n; rr += NW) {
            // v_rr and w_rr from the lane that holds column rr (rr is wave-uniform)
            const int src = rr - k - 1;
            const double2 vr = c_make(wg_lane_read(vc.x, src), wg_lane_read(vc.y, src));
            const double2 wr = c_make(wg_lane_read(wc.x, src), wg_lane_read(wc.y, src));
            if (c < n) {
                const double2 x = c_rank2c(P[rr * n + c], vr, wc, wr, vc);
                P[rr * n + c] = x;
                if (lane == 0 && rr > k + 1) {
                    S.xv[rr] = x;
                    if (rr > k + 2) nrm_part = fma(x.x, x.x, fma(x.y, x.y, nrm_part));
                }
            }
        }
        if (lane == 0) S.red[w] = nrm_part;
        __syncthreads();
    }
    if (tid == 0) {
        S.d[n - 1] = P[(n - 1) * n + (n - 1)].x;
        S.e[n - 1] = 0.0;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// step 2b: eigenvalues (S.lam ascending) by Sturm counts with safeguarded
// Newton steps: tpe threads per eigenvalue keep one bracket lo <= lambda_j < hi
// (with the counts at its ends).  Per pass, while lambda_j is not alone in the
// bracket the threads count at tpe equally spaced interior points
// (multisection); once it is, thread 0 takes the Newton point x - 1/S of the
// previous pass, S = d/dx log|det(T - x I)| from the derivative recurrence
// q_i' = -1 + e_{i-1}^2 q_{i-1}' / q_{i-1}^2, and the others split the bracket.
// A Newton step below the tolerance is accepted only after a pass whose counts
// at c -/+ 2 tol bracket lambda_j, so the counts decide the result as in
// bisection.
// ---------------------------------------------------------------------------
__device__ void wg_bisect(WgLds& S, int n, double& pivmin_out, double& span_out) {
    const int tid = threadIdx.x;
    double lo_i = 1e300, hi_i = -1e300, emax = 0.0;
    for (int i = tid; i < n; i += kWgThreads) {
        const double rad = fabs(S.e[i]) + (i > 0 ? fabs(S.e[i - 1]) : 0.0);
        lo_i = fmin(lo_i, S.d[i] - rad);
        hi_i = fmax(hi_i, S.d[i] + rad);
        emax = fmax(emax, fabs(S.e[i]));
    }
    const double glo = wg_min(lo_i, S.red);
    const double ghi = wg_max(hi_i, S.red);
    const double em = wg_max(emax, S.red);
    const double pivmin = 1e-290 * fmax(1.0, em * em);
    pivmin_out = pivmin;
    span_out = fmax(fabs(glo), fabs(ghi));
    auto rcp = [](double q) {
        const double r = __builtin_amdgcn_rcp(q);
        return fma(r, fma(-q, r, 1.0), r);
    };
    int np2 = 1;
    while (np2 < n) np2 <<= 1;
    const int tpe = kWgThreads / np2;  // threads per eigenvalue (>= 2, divides 64)
    const int j = tid / tpe, q = tid - (tid / tpe) * tpe;
    const int base = (tid & 63) - q;  // first lane of the group
    const double tol = 4.0 * 2.220446049250313e-16 * span_out + 1e-300;
    double lo = glo, hi = ghi, cand = 0.0, lam = ghi;
    int clo = 0, chi = n;
    bool done = j >= n, has = false, ver = false;
    for (int pass = 0; pass < 160; ++pass) {
        if (__ballot(!done) == 0ull) break;  // per wavefront: whole groups
        const bool iso = (clo == j) && (chi == j + 1);
        const double w = hi - lo;
        double x;
        if (ver)
            x = (q == 0) ? cand - 2.0 * tol : ((q == 1) ? cand + 2.0 * tol : lo + w * (double)q / (double)tpe);
        else if (iso && has)
            x = (q == 0) ? cand : lo + w * (double)q / (double)tpe;
        else
            x = lo + w * (double)(q + 1) / (double)(tpe + 1);
        const bool need_d = __ballot(!done && iso && !ver) != 0ull;
        int cnt = 0;
        double sd = 0.0;
        if (need_d) {
            double qv = 1.0, qd = 0.0, e2prev = 0.0;
            for (int i = 0; i < n; ++i) {
                const double rq = rcp(qv);
                sd = fma(qd, rq, sd);  // q'_{i-1} / q_{i-1}
                const double t = e2prev * rq;
                double qi = (S.d[i] - x) - t;
                if (fabs(qi) < pivmin) qi = -pivmin;
                qd = fma(t * rq, qd, -1.0);
                cnt += (qi < 0.0) ? 1 : 0;
                qv = qi;
                e2prev = S.e[i] * S.e[i];
            }
            sd = fma(qd, rcp(qv), sd);
        } else {
            double qv = 1.0, e2prev = 0.0;
            for (int i = 0; i < n; ++i) {
                double qi = fma(-e2prev, rcp(qv), S.d[i] - x);
                if (fabs(qi) < pivmin) qi = -pivmin;
                cnt += (qi < 0.0) ? 1 : 0;
                qv = qi;
                e2prev = S.e[i] * S.e[i];
            }
        }
        // this thread's Newton point
        const double nx = need_d ? x - 1.0 / sd : 0.0;
        const double nst = fabs(nx - x);
        // every thread of the group applies all tpe points in the same order
        const int c0 = __shfl(cnt, base, 64), c1 = __shfl(cnt, base + 1, 64);
        const bool verified = ver && c0 <= j && c1 > j;
        for (int p = 0; p < tpe; ++p) {
            const double xp = __shfl(x, base + p, 64);
            const int cp = __shfl(cnt, base + p, 64);
            if (!done && !verified) {
                if (cp <= j && xp > lo) {
                    lo = xp;
                    clo = cp;
                }
                if (cp > j && xp < hi) {
                    hi = xp;
                    chi = cp;
                }
            }
        }
        bool found = false;
        double best = 0.0, bst = 0.0;
        if (need_d) {
            for (int p = 0; p < tpe; ++p) {
                const double np_ = __shfl(nx, base + p, 64);
                const double sp = __shfl(nst, base + p, 64);
                const bool in = (np_ >= lo - tol) && (np_ <= hi + tol);
                if (in && (!found || sp < bst)) {
                    found = true;
                    best = np_;
                    bst = sp;
                }
            }
        }
        if (done) continue;
        if (verified) {
            done = true;
            lam = cand;
            continue;
        }
        const bool was_ver = ver;
        ver = false;
        has = false;
        if (found && !was_ver) {
            cand = fmin(fmax(best, lo), hi);
            if ((clo == j) && (chi == j + 1) && bst <= tol)
                ver = true;
            else
                has = (best > lo) && (best < hi);
        }
        if (!ver && hi - lo <= tol) {
            done = true;
            lam = 0.5 * (lo + hi);
        }
    }
    if (!done) lam = 0.5 * (lo + hi);
    if (q == 0 && j < n) S.lam[j] = lam;
    __syncthreads();
}

// ---------------------------------------------------------------------------
// step 2c: eigenvectors of T by twisted factorisations, Z -> U (real parts)
// thread j owns eigenvector j; pivots go to DPM in [i][j] order (coalesced)
// ---------------------------------------------------------------------------
__device__ void wg_twisted(WgLds& S, const WgScratch& X, int n, double pivmin, double* __restrict__ R,
                           size_t r_doubles) {
    // one pivot array per eigenvector in the LDS region R, G eigenvectors at a time
    // (piv[i][t] at R[i G + t]: consecutive threads, consecutive words).  Pass 1 stores
    // the forward pivots dp_i; pass 2 runs the backward pivots dm_i without storing them
    // and picks the twist index r; pass 3 recomputes dm_i for i > r into the slots of
    // dp_i, which the solve above r no longer needs.
    const int Gmax = (int)(r_doubles / (size_t)n);
    const int G = Gmax < n ? Gmax : n;
    // reciprocal: hardware estimate and one Newton step (|q| >= pivmin keeps it finite)
    auto rcp = [](double q) {
        const double r0 = __builtin_amdgcn_rcp(q);
        return fma(r0, fma(-q, r0, 1.0), r0);
    };
    for (int g0 = 0; g0 < n; g0 += G) {
        const int t = threadIdx.x, j = g0 + t;
        if (t < G && j < n) {
            const double lam = S.lam[j];
            double* piv = R + t;
            double qv = 1.0, e2prev = 0.0;
            for (int i = 0; i < n; ++i) {
                double qi = (S.d[i] - lam) - e2prev * rcp(qv);
                if (fabs(qi) < pivmin) qi = -pivmin;
                piv[i * G] = qi;
                qv = qi;
                e2prev = S.e[i] * S.e[i];
            }
            qv = 1.0;
            int r = 0;
            double best = 1e308, gam = 0.0;
            for (int i = n - 1; i >= 0; --i) {
                double qi = (S.d[i] - lam) - ((i < n - 1) ? S.e[i] * S.e[i] * rcp(qv) : 0.0);
                if (fabs(qi) < pivmin) qi = -pivmin;
                qv = qi;
                const double g = piv[i * G] + qi - (S.d[i] - lam);
                if (fabs(g) < best) {
                    best = fabs(g);
                    gam = g;
                    r = i;
                }
            }
            qv = 1.0;
            for (int i = n - 1; i > r; --i) {
                double qi = (S.d[i] - lam) - ((i < n - 1) ? S.e[i] * S.e[i] * rcp(qv) : 0.0);
                if (fabs(qi) < pivmin) qi = -pivmin;
                piv[i * G] = qi;
                qv = qi;
            }
            double nrm = 1.0;
            double z = 1.0;
            for (int i = r - 1; i >= 0; --i) {
                z = -(S.e[i] * rcp(piv[i * G])) * z;
                piv[i * G] = z;  // the pivot is spent: keep z_i in its place
                nrm += z * z;
            }
            z = 1.0;
            for (int i = r + 1; i < n; ++i) {
                z = -(S.e[i - 1] * rcp(piv[i * G])) * z;
                piv[i * G] = z;
                nrm += z * z;
            }
            const double inv = 1.0 / sqrt(nrm);
            for (int i = 0; i < n; ++i) {
                const double zi = (i == r) ? 1.0 : piv[i * G];
                X.U[(long long)i * n + j] = c_make(zi * inv, 0.0);
            }
            // (T - lam) z = gam e_r with z_r = 1: Rayleigh-quotient correction
            S.E[j] = lam + gam / nrm;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// step 2c': implicit QL with accumulated rotations (clustered spectra)
// every thread follows the same scalar chain (d, e in LDS); thread r owns row r of Z
// ---------------------------------------------------------------------------
__device__ bool wg_ql(WgLds& S, double2* __restrict__ Z, int n, int max_iter) {
    const int tid = threadIdx.x;
    for (int e = tid; e < n * n; e += kWgThreads) {
        const int i = e / n, j = e - (e / n) * n;
        Z[e] = c_make(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    bool ok = true;
    double f = 0.0, tst1 = 0.0;
    for (int l = 0; l < n && ok; ++l) {
        int iter = 0;
        tst1 = fmax(tst1, fabs(S.d[l]) + fabs(S.e[l]));
        for (;;) {
            int m = l;
            while (m < n - 1 && !(tst1 + fabs(S.e[m]) == tst1)) ++m;
            if (m == l) break;
            if (++iter > max_iter || !isfinite(tst1)) {
                ok = false;
                break;
            }
            const double g0 = S.d[l], el = S.e[l];
            double p = (S.d[l + 1] - g0) / (2.0 * el);
            double r = sqrt(p * p + 1.0);
            const double pr = p + copysign(r, p);
            const double new_dl = el / pr, dl1 = el * pr;
            double h = g0 - new_dl;
            __syncthreads();
            for (int i = l + 2 + tid; i < n; i += kWgThreads) S.d[i] -= h;
            if (tid == 0) {
                S.d[l] = new_dl;
                S.d[l + 1] = dl1;
            }
            f += h;
            __syncthreads();
            p = S.d[m];
            double c = 1.0, c2 = 1.0, c3 = 1.0, s = 0.0, s2 = 0.0;
            const double el1 = S.e[l + 1];
            // the chain: every thread computes it from the unmodified d, e;
            // thread 0 records the new values aside and the rotations
            for (int i = m - 1; i >= l; --i) {
                c3 = c2;
                c2 = c;
                s2 = s;
                const double ei = S.e[i], di = S.d[i];
                const double g = c * ei;
                h = c * p;
                r = sqrt(p * p + ei * ei);
                const double e_ip1 = s * r;
                const double inv = 1.0 / r;
                s = ei * inv;
                c = p * inv;
                p = c * di - s * g;
                const double d_ip1 = h + s * (c * g + s * di);
                if (tid == 0) {
                    S.en[i + 1] = e_ip1;
                    S.dn[i + 1] = d_ip1;
                    S.cs[2 * i] = c;
                    S.cs[2 * i + 1] = s;
                }
            }
            __syncthreads();
            for (int i = l + 1 + tid; i <= m; i += kWgThreads) {
                S.e[i] = S.en[i];
                S.d[i] = S.dn[i];
            }
            if (tid == 0) {
                const double pp = -s * s2 * c3 * el1 * el / dl1;
                S.e[l] = s * pp;
                S.d[l] = c * pp;
            }
            __syncthreads();
            for (int row = tid; row < n; row += kWgThreads) {
                double carry = Z[row * n + m].x;
                for (int i = m - 1; i >= l; --i) {
                    const double ci = S.cs[2 * i], si = S.cs[2 * i + 1];
                    const double zi = Z[row * n + i].x;
                    Z[row * n + i + 1].x = si * zi + ci * carry;
                    carry = ci * zi - si * carry;
                }
                Z[row * n + l].x = carry;
            }
            __syncthreads();
        }
        __syncthreads();
        if (tid == 0) S.d[l] += f;
        __syncthreads();
    }
    for (int i = tid; i < n; i += kWgThreads) {
        S.E[i] = S.d[i];
        if (!isfinite(S.d[i])) ok = false;
    }
    __syncthreads();
    return ok;
}

// ---------------------------------------------------------------------------
// step 2d: U <- H_0 ... H_{n-2} U with U's column c in registers, four threads
// per column (rows 4 jj + g), 64 columns per pass (one pass for n <= 64, two
// for n <= 128), the reflectors staged into LDS sixteen columns at a time, and
// groups of four row slots that lie above the reflector skipped by a
// wave-uniform test.  No global traffic but one read and one write of U.
// ---------------------------------------------------------------------------
template <int NR>
__device__ void wg_backtransform_reg(WgLds& S, const double2* __restrict__ P, double2* __restrict__ U,
                                     int n) {
    // NR = 64 or 128 rows at most: four threads per column (a DPP quad), each holding the
    // rows g, g + 4, ... of its column in registers; 64 columns per pass
    constexpr int G = 4, RJ = NR / G, KC = 16;
    const int tid = threadIdx.x;
    double2* V = S.ta;  // [KC][NR]: reflector columns k0 .. k0+KC-1 (the LDS scratch region)
    for (int c0 = 0; c0 < n; c0 += kWgThreads / G) {
        const int c = c0 + (tid >> 2), g = tid & 3;
        const bool act = c < n;
        double2 u[RJ];
#pragma unroll
        for (int jj = 0; jj < RJ; ++jj) {
            const int r = G * jj + g;
            u[jj] = (act && r < n) ? U[r * n + c] : c_make(0.0, 0.0);
        }
        for (int k1 = n - 1; k1 > 0; k1 -= KC) {
            const int k0 = (k1 - KC > 0) ? k1 - KC : 0;  // this chunk: reflectors k0 .. k1-1
            __syncthreads();
            for (int e = tid; e < (k1 - k0) * NR; e += kWgThreads) {
                const int kk = e / NR, r = e - (e / NR) * NR;
                const int k = k0 + kk;
                V[kk * NR + r] = (r > k && r < n) ? P[r * n + k] : c_make(0.0, 0.0);
            }
            __syncthreads();
            for (int k = k1 - 1; k >= k0; --k) {
                const double2 tau = S.tau[k];
                if (tau.x == 0.0 && tau.y == 0.0) continue;
                const double2* v = V + (k - k0) * NR;
                double2 y = c_make(0.0, 0.0);
#pragma unroll
                for (int gq = 0; gq < RJ / 4; ++gq) {
                    if (16 * gq + 15 > k) {
#pragma unroll
                        for (int t = 0; t < 4; ++t) y = c_fmac(v[G * (4 * gq + t) + g], u[4 * gq + t], y);
                    }
                }
                // the column's four threads are a DPP quad
                y.x += __builtin_amdgcn_update_dpp(0.0, y.x, 0xB1, 0xF, 0xF, false);
                y.y += __builtin_amdgcn_update_dpp(0.0, y.y, 0xB1, 0xF, 0xF, false);
                y.x += __builtin_amdgcn_update_dpp(0.0, y.x, 0x4E, 0xF, 0xF, false);
                y.y += __builtin_amdgcn_update_dpp(0.0, y.y, 0x4E, 0xF, 0xF, false);
                const double2 ty = c_mul(tau, y);
#pragma unroll
                for (int gq = 0; gq < RJ / 4; ++gq) {
                    if (16 * gq + 15 > k) {
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const int jj = 4 * gq + t;
                            u[jj] = c_fnma(v[G * jj + g], ty, u[jj]);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int jj = 0; jj < RJ; ++jj) {
            const int r = G * jj + g;
            if (act && r < n) U[r * n + c] = u[jj];
        }
    }
    __syncthreads();
}

// C = A B (n x n, complex) on the FP64 matrix cores; A and B come from the
// element functions LA(i, k), LB(k, j) (global scratch, transposes and
// conjugates folded in), C must not alias them.  The four wavefronts take
// 32 x 32 blocks of C in turn; a block is 2 x 2 tiles of v_mfma_f64_16x16x4
// with separate real and imaginary accumulators (four real products per
// complex one).  Lane (g, c) = (lane / 16, lane % 16) supplies A[16 t + c][k]
// and B[k][16 t + c] for k = 4 kk + g; elements past n are zero.
typedef double wg_v4d __attribute__((ext_vector_type(4)));
__device__ __forceinline__ wg_v4d wg_mfma16(double a, double b, wg_v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <class FA, class FB>
__device__ void wg_gemm_mfma(WgLds& S, double2* __restrict__ C, int n, FA LA, FB LB) {
    (void)S;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int nb = (n + 31) >> 5;  // 32 x 32 blocks per dimension
    const int nk = (n + 3) >> 2;   // k-steps of four
    const wg_v4d zero = {0.0, 0.0, 0.0, 0.0};
    for (int blk = wv; blk < nb * nb; blk += kWgThreads / 64) {
        const int bi = blk / nb, bj = blk - (blk / nb) * nb;
        wg_v4d cr[2][2], ci[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                cr[a][b] = zero;
                ci[a][b] = zero;
            }
#pragma unroll 2
        for (int kk = 0; kk < nk; ++kk) {
            const int k = 4 * kk + g;
            double2 av[2], bv[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int row = 32 * bi + 16 * t + c, col = 32 * bj + 16 * t + c;
                av[t] = (row < n && k < n) ? LA(row, k) : c_make(0.0, 0.0);
                bv[t] = (k < n && col < n) ? LB(k, col) : c_make(0.0, 0.0);
            }
#pragma unroll
            for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                for (int tj = 0; tj < 2; ++tj) {
                    cr[ti][tj] = wg_mfma16(av[ti].x, bv[tj].x, cr[ti][tj]);
                    cr[ti][tj] = wg_mfma16(-av[ti].y, bv[tj].y, cr[ti][tj]);
                    ci[ti][tj] = wg_mfma16(av[ti].x, bv[tj].y, ci[ti][tj]);
                    ci[ti][tj] = wg_mfma16(av[ti].y, bv[tj].x, ci[ti][tj]);
                }
        }
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int tj = 0; tj < 2; ++tj)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = 32 * bi + 16 * ti + g + 4 * q, col = 32 * bj + 16 * tj + c;
                    if (row < n && col < n) C[row * n + col] = c_make(cr[ti][tj][q], ci[ti][tj][q]);
                }
    }
    __syncthreads();
}

// The same product through 32 x 32 LDS tiles on the vector ALUs (LA and LB as
// above).  Used for n > 64: there the matrix-core version measured slower in
// the adjoint (its operands come uncoalesced from a scratch slice that no
// longer fits in the caches, and its accumulators cost the kernel its second
// wavefront per SIMD).
template <class FA, class FB>
__device__ void wg_gemm_tiles(WgLds& S, double2* __restrict__ C, int n, FA LA, FB LB) {
    const int tid = threadIdx.x;
    const int ti = tid >> 4, tj = tid & 15;  // 2 x 2 outputs per thread
    const int nt = (n + kTile - 1) / kTile;
    for (int bi = 0; bi < nt; ++bi)
        for (int bj = 0; bj < nt; ++bj) {
            double2 acc[2][2];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) acc[a][b] = c_make(0.0, 0.0);
            for (int bk = 0; bk < nt; ++bk) {
                for (int e = tid; e < kTile * kTile; e += kWgThreads) {
                    const int r = e / kTile, c = e - (e / kTile) * kTile;
                    const int gi = bi * kTile + r, gk = bk * kTile + c;
                    S.ta[r * (kTile + 1) + c] = (gi < n && gk < n) ? LA(gi, gk) : c_make(0.0, 0.0);
                    const int gk2 = bk * kTile + r, gj = bj * kTile + c;
                    S.tb[r * (kTile + 1) + c] = (gk2 < n && gj < n) ? LB(gk2, gj) : c_make(0.0, 0.0);
                }
                __syncthreads();
                for (int kk = 0; kk < kTile; ++kk) {
                    const double2 a0 = S.ta[(2 * ti) * (kTile + 1) + kk];
                    const double2 a1 = S.ta[(2 * ti + 1) * (kTile + 1) + kk];
                    const double2 b0 = S.tb[kk * (kTile + 1) + 2 * tj];
                    const double2 b1 = S.tb[kk * (kTile + 1) + 2 * tj + 1];
                    acc[0][0] = c_fma(a0, b0, acc[0][0]);
                    acc[0][1] = c_fma(a0, b1, acc[0][1]);
                    acc[1][0] = c_fma(a1, b0, acc[1][0]);
                    acc[1][1] = c_fma(a1, b1, acc[1][1]);
                }
                __syncthreads();
            }
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    const int gi = bi * kTile + 2 * ti + a, gj = bj * kTile + 2 * tj + b;
                    if (gi < n && gj < n) C[gi * n + gj] = acc[a][b];
                }
        }
    __syncthreads();
}

// C = A B with C n x n and an inner dimension nk (complex) on the FP64 matrix cores,
// operands staged through LDS.  C is taken in 64 x 64 macro tiles; per panel of
// kWgKT inner indices the workgroup copies A[64 rows][kWgKT] and B[kWgKT][64 cols]
// into the LDS scratch region with coalesced global reads (A_IFAST: LA(i, k) is
// contiguous in i in memory, else in k; B_KFAST: LB(k, j) contiguous in k, else in
// j), then each wavefront accumulates its 32 x 32 block as 2 x 2 tiles of
// v_mfma_f64_16x16x4 with separate real and imaginary accumulators (four real
// products per complex one; eight independent accumulators).  Rows padded by one
// element keep the operand reads free of bank conflicts.
constexpr int kWgKT = 16;
constexpr int kWgLdA = kWgKT + 1, kWgLdB = 64 + 1;
template <bool A_IFAST, bool B_KFAST, class FA, class FB>
__device__ void wg_gemm_lds(WgLds& S, double2* __restrict__ C, int n, int nk, FA LA, FB LB) {
    double2* As = S.ta;                // [64][kWgLdA]
    double2* Bs = S.ta + 64 * kWgLdA;  // [kWgKT][kWgLdB]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int wr = w >> 1, wc = w & 1;
    const wg_v4d zero = {0.0, 0.0, 0.0, 0.0};
    const int nmt = (n + 63) >> 6;
    for (int mt = 0; mt < nmt * nmt; ++mt) {
        const int i0 = 64 * (mt / nmt), j0 = 64 * (mt - (mt / nmt) * nmt);
        wg_v4d cr[2][2], ci[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                cr[a][b] = zero;
                ci[a][b] = zero;
            }
        for (int kb = 0; kb < nk; kb += kWgKT) {
            // the tiles' elements of this thread: every load issued first (indices
            // clamped into the matrices, so each is valid), zeros outside stored after
            constexpr int PER = 64 * kWgKT / kWgThreads;
            double2 ta[PER], tb[PER];
#pragma unroll
            for (int r = 0; r < PER; ++r) {
                const int e = tid + r * kWgThreads;
                const int ii = A_IFAST ? (e & 63) : (e / kWgKT);
                const int kk = A_IFAST ? (e >> 6) : (e - (e / kWgKT) * kWgKT);
                ta[r] = LA(min(i0 + ii, n - 1), min(kb + kk, nk - 1));
                const int jj = B_KFAST ? (e / kWgKT) : (e & 63);
                const int k2 = B_KFAST ? (e - (e / kWgKT) * kWgKT) : (e >> 6);
                tb[r] = LB(min(kb + k2, nk - 1), min(j0 + jj, n - 1));
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < PER; ++r) {
                const int e = tid + r * kWgThreads;
                const int ii = A_IFAST ? (e & 63) : (e / kWgKT);
                const int kk = A_IFAST ? (e >> 6) : (e - (e / kWgKT) * kWgKT);
                As[ii * kWgLdA + kk] = (i0 + ii < n && kb + kk < nk) ? ta[r] : c_make(0.0, 0.0);
                const int jj = B_KFAST ? (e / kWgKT) : (e & 63);
                const int k2 = B_KFAST ? (e - (e / kWgKT) * kWgKT) : (e >> 6);
                Bs[k2 * kWgLdB + jj] = (kb + k2 < nk && j0 + jj < n) ? tb[r] : c_make(0.0, 0.0);
            }
            __syncthreads();
#pragma unroll
            for (int k4 = 0; k4 < kWgKT / 4; ++k4) {
                double2 av[2], bv[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    av[t] = As[(32 * wr + 16 * t + c) * kWgLdA + 4 * k4 + g];
                    bv[t] = Bs[(4 * k4 + g) * kWgLdB + 32 * wc + 16 * t + c];
                }
#pragma unroll
                for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                    for (int tj = 0; tj < 2; ++tj) cr[ti][tj] = wg_mfma16(av[ti].x, bv[tj].x, cr[ti][tj]);
#pragma unroll
                for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                    for (int tj = 0; tj < 2; ++tj) ci[ti][tj] = wg_mfma16(av[ti].x, bv[tj].y, ci[ti][tj]);
#pragma unroll
                for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                    for (int tj = 0; tj < 2; ++tj) cr[ti][tj] = wg_mfma16(-av[ti].y, bv[tj].y, cr[ti][tj]);
#pragma unroll
                for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                    for (int tj = 0; tj < 2; ++tj) ci[ti][tj] = wg_mfma16(av[ti].y, bv[tj].x, ci[ti][tj]);
            }
        }
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int tj = 0; tj < 2; ++tj)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = i0 + 32 * wr + 16 * ti + g + 4 * q, col = j0 + 32 * wc + 16 * tj + c;
                    if (row < n && col < n) C[row * n + col] = c_make(cr[ti][tj][q], ci[ti][tj][q]);
                }
    }
    __syncthreads();
}

// C = A B, n x n by n x n, for the orientation flags of wg_gemm_lds
template <bool A_IFAST, bool B_KFAST, class FA, class FB>
__device__ __forceinline__ void wg_gemm(WgLds& S, double2* __restrict__ C, int n, FA LA, FB LB) {
    wg_gemm_lds<A_IFAST, B_KFAST>(S, C, n, n, LA, LB);
}

// Steps 1-3: E (S.E), U, and A = U^+ v_x U in X.VX, B = U^+ v_y U in X.VY.
template <bool SMALL>
__device__ bool wg_eigen_velocities(WgLds& S, const WgScratch& X, const ModelDev& md,
                                    const double2* __restrict__ T0, const double2* __restrict__ T1,
                                    const int* __restrict__ r0, int i0, int max_iter) {
    const int n = md.n;
    wg_build(S, X, md, T0, T1, r0, i0);
    if constexpr (SMALL) {
        // on an LDS copy of the matrix (see kWgSmallLds)
        unsigned char* base = reinterpret_cast<unsigned char*>(&S);
        double2* Pl = reinterpret_cast<double2*>(base + offsetof(WgLds, lam));
        double2* part = reinterpret_cast<double2*>(base + kWgSmallLds - kWgSmallPart);
        for (int e = threadIdx.x; e < n * n; e += kWgThreads) Pl[e] = X.P[e];
        __syncthreads();
        wg_tridiag_cols(S, Pl, n, part);
        for (int e = threadIdx.x; e < n * n; e += kWgThreads) X.P[e] = Pl[e];
        __syncthreads();
    } else {
        wg_tridiag_packed(S, X.P, n, reinterpret_cast<double2*>(wg_region(S)));
    }
    double pivmin, span;
    wg_bisect(S, n, pivmin, span);
    int close = 0;
    for (int j = threadIdx.x; j < n - 1; j += kWgThreads)
        if (S.lam[j + 1] - S.lam[j] < kWgClusterGap * span) close = 1;
    if (threadIdx.x == 0) S.flag = 0;
    __syncthreads();
    if (close) S.flag = 1;
    __syncthreads();
    bool ok = true;
    if (S.flag == 0 && max_iter > 1) {
        wg_twisted(S, X, n, pivmin, wg_region(S), wg_region_doubles<SMALL>());
        for (int j = threadIdx.x; j < n; j += kWgThreads)
            if (!isfinite(S.E[j])) ok = false;
    } else {
        ok = wg_ql(S, X.U, n, max_iter);
    }
    wg_backtransform_reg<SMALL ? 64 : 128>(S, X.P, X.U, n);
    const double2* U = X.U;
    double2* W = X.W;
    double2* VX = X.VX;
    double2* VY = X.VY;
    wg_gemm<false, false>(S, W, n, [=](int i, int k) { return VX[i * n + k]; },
            [=](int k, int j) { return U[k * n + j]; });
    wg_gemm<true, false>(S, VX, n, [=](int i, int k) { return c_conj(U[k * n + i]); },
            [=](int k, int j) { return W[k * n + j]; });
    wg_gemm<false, false>(S, W, n, [=](int i, int k) { return VY[i * n + k]; },
            [=](int k, int j) { return U[k * n + j]; });
    wg_gemm<true, false>(S, VY, n, [=](int i, int k) { return c_conj(U[k * n + i]); },
            [=](int k, int j) { return W[k * n + j]; });
    return ok;
}

// ---------------------------------------------------------------------------
// k_forward_wg
// ---------------------------------------------------------------------------
// SMALL (n <= 64): LDS-resident reduction, register back-transformation, matrix-core GEMMs.
// TENSOR: also C = U^+ v_z U (in the pivot region, dead after the eigenvectors) and
// D = U^+ Js_x U (in the K region, unused by the forward), four curvatures per band and
// four Fermi sums per level, [slot][4][nF].
template <bool SMALL, bool TENSOR>
__global__ __launch_bounds__(kWgThreads, SMALL ? 2 : 1) void k_forward_wg(WgLaunch a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    WgLds& S = *reinterpret_cast<WgLds*>(smem_raw);
    const double eta2 = a.eta * a.eta;
    constexpr int NC = TENSOR ? 4 : 1;
    const WgScratch X = wg_scratch(reinterpret_cast<double2*>(a.scratch), a.slot_elems, blockIdx.x);
    const double2* tbuf = reinterpret_cast<const double2*>(a.tbuf);
    double2* VZ = reinterpret_cast<double2*>(X.DPM);
    double2* JS = reinterpret_cast<double2*>(X.K);
    int probe = 0;
    for (int par = 0;; par ^= 1) {
        if (threadIdx.x == 0) S.unit[par] = queue_take(a.queue, a.item_count, probe);
        __syncthreads();
        const int item = S.unit[par];
        if (item < 0) break;
        const BlockItem it = a.tb.blocks[a.item_begin + item];
        const ModelDev md = a.tb.models[it.model];
        const int n = md.n;
        const long long nn = (long long)n * n;
        const double2* T0 = tbuf + it.tbuf_off;
        const double2* T1 = T0 + (long long)md.nR0 * nn;
        const double2* T2 = T1 + (long long)md.nR0 * nn;
        const int* r0 = a.tb.r0val + md.r0_first;
        const double* ef = a.e_fermi + md.f_off;
        const double* spin = (TENSOR && a.spin) ? a.spin + md.orb_off : nullptr;
        double* part = a.partial + (long long)it.slot * a.nF * NC;
        for (int kk = 0; kk < it.count; ++kk) {
            const bool ok = wg_eigen_velocities<SMALL>(S, X, md, T0, T1, r0, it.i0 + kk, a.max_iter);
            if (!ok) atomicOr(a.status, kStatNoConv);
            if constexpr (TENSOR) {
                wg_build_tensor(S, md, T0, T2, r0, it.i0 + kk, spin, VZ, JS);
                const double2* U = X.U;
                double2* W = X.W;
                wg_gemm<false, false>(S, W, n, [=](int i, int k) { return VZ[i * n + k]; },
                        [=](int k, int j) { return U[k * n + j]; });
                wg_gemm<true, false>(S, VZ, n, [=](int i, int k) { return c_conj(U[k * n + i]); },
                        [=](int k, int j) { return W[k * n + j]; });
                if (spin) {
                    wg_gemm<false, false>(S, W, n, [=](int i, int k) { return JS[i * n + k]; },
                            [=](int k, int j) { return U[k * n + j]; });
                    wg_gemm<true, false>(S, JS, n, [=](int i, int k) { return c_conj(U[k * n + i]); },
                            [=](int k, int j) { return W[k * n + j]; });
                }
            }
            // Omega_i = -2 sum_{m != i} Im(P_im Q_mi) g(E_i - E_m) per operator pair
            auto curv = [&](const double2* P, const double2* Q, int i) {
                double om = 0.0;
                const double ei = S.E[i];
                for (int m = 0; m < n; ++m) {
                    if (m == i) continue;
                    const double de = ei - S.E[m];
                    const double den = de * de + eta2;
                    if (den == 0.0) continue;
                    const double2 x = P[i * n + m], y = Q[m * n + i];
                    om += (x.x * y.y + x.y * y.x) / den;
                }
                return -2.0 * om;
            };
            for (int i = threadIdx.x; i < n; i += kWgThreads) {
                S.Om[i] = curv(X.VX, X.VY, i);
                if constexpr (TENSOR) {
                    S.Om2[0][i] = curv(X.VY, VZ, i);
                    S.Om2[1][i] = curv(VZ, X.VX, i);
                    S.Om2[2][i] = spin ? curv(JS, X.VY, i) : 0.0;
                }
            }
            __syncthreads();
            for (int j = threadIdx.x; j < a.nF; j += kWgThreads) {
                const double efj = ef[j];
                double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
                for (int b = 0; b < n; ++b) {
                    const double f = occupation(S.E[b], efj, a.kT);
                    s0 += f * S.Om[b];
                    if constexpr (TENSOR) {
                        s1 += f * S.Om2[0][b];
                        s2 += f * S.Om2[1][b];
                        s3 += f * S.Om2[2][b];
                    }
                }
                if (!isfinite(s0 + s1 + s2 + s3)) atomicOr(a.status, kStatNonFinite);
                part[j] = (kk == 0) ? s0 : part[j] + s0;
                if constexpr (TENSOR) {
                    part[a.nF + j] = (kk == 0) ? s1 : part[a.nF + j] + s1;
                    part[2 * a.nF + j] = (kk == 0) ? s2 : part[2 * a.nF + j] + s2;
                    part[3 * a.nF + j] = (kk == 0) ? s3 : part[3 * a.nF + j] + s3;
                }
            }
            __syncthreads();
        }
    }
}

// phi(x) = sum_j sbar_j f_j(x) and its derivative
__device__ __forceinline__ void wg_phi_at(double x, const double* __restrict__ ef,
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

// ---------------------------------------------------------------------------
// k_adjoint_wg: reverse mode per k-point (the formulas of the one-wavefront
// adjoint in kubo_wave.hip); stores each k-point's Hbar, vbar_x, vbar_y, from
// which k_pacc forms the block's pencil partials.
// ---------------------------------------------------------------------------
template <bool SMALL>
__global__ __launch_bounds__(kWgThreads, SMALL ? 2 : 1) void k_adjoint_wg(WgLaunch a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    WgLds& S = *reinterpret_cast<WgLds*>(smem_raw);
    const double eta2 = a.eta * a.eta;
    const double scl = (a.kT > 0.0) ? fmin(a.eta, a.kT) : a.eta;
    const double delta = 1e-5 * scl;
    const WgScratch X = wg_scratch(reinterpret_cast<double2*>(a.scratch), a.slot_elems, blockIdx.x);
    const double2* tbuf = reinterpret_cast<const double2*>(a.tbuf);
    const int units = a.item_count * a.unit_parts;
    int probe = 0;
    for (int par = 0;; par ^= 1) {
        if (threadIdx.x == 0) S.unit[par] = queue_take(a.queue, units, probe);
        __syncthreads();
        const int unit = S.unit[par];
        if (unit < 0) break;
        const int item = unit / a.unit_parts;
        const int kk0 = (unit - item * a.unit_parts) * a.unit_k;
        const BlockItem it = a.tb.blocks[a.item_begin + item];
        const int kk1 = min(it.count, kk0 + a.unit_k);
        const ModelDev md = a.tb.models[it.model];
        const int n = md.n;
        const long long nn = (long long)n * n;
        const double2* T0 = tbuf + it.tbuf_off;
        const double2* T1 = T0 + (long long)md.nR0 * nn;
        const int* r0 = a.tb.r0val + md.r0_first;
        const double* ef = a.e_fermi + md.f_off;
        const double* sb = a.sbar + md.f_off;
        const double invN = 1.0 / (double)md.Nk;
        for (int kk = kk0; kk < kk1; ++kk) {
            const bool ok = wg_eigen_velocities<SMALL>(S, X, md, T0, T1, r0, it.i0 + kk, a.max_iter);
            if (!ok) atomicOr(a.status, kStatNoConv);
            const double2* A = X.VX;
            const double2* B = X.VY;
            for (int b = threadIdx.x; b < n; b += kWgThreads) {
                double p, d;
                wg_phi_at(S.E[b], ef, sb, a.nF, a.kT, p, d);
                S.phi[b] = p;
                S.dphi[b] = d;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < n * n; e += kWgThreads) {
                const int m = e / n, q = e - (e / n) * n;
                double k = 0.0;
                if (m != q) {
                    const double de = S.E[m] - S.E[q];
                    k = (S.phi[m] - S.phi[q]) / (de * de + eta2);
                }
                X.K[e] = k;
            }
            __syncthreads();
            // Hbar'_mq = X_mq / (E_m - E_q) with X = (i/N)(D + D^+), D = (K o B) A - (K o A) B
            // and D^+ = B (K o A) - A (K o B) (K is real and antisymmetric, A and B are
            // Hermitian): two products with an inner dimension of 2n, [K o B, -K o A][A; B]
            // into W and [A, B][-K o B; K o A] into P.  On the diagonal and for pairs closer
            // than delta the divided-difference limit (i/N) sum_p dK(x, E_p)/dx
            // (B_mp A_pq - A_mp B_pq) at x = (E_m + E_q)/2.  Hbar' goes to HB (the pivot
            // region, dead by now).
            const double2* U = X.U;
            double2* P = X.P;
            double2* W = X.W;
            double2* VX = X.VX;
            double2* VY = X.VY;
            const double* K = X.K;
            double2* HB = reinterpret_cast<double2*>(X.DPM);
            wg_gemm_lds<false, false>(S, W, n, 2 * n,
                    [=](int i, int k) {
                        return k < n ? c_scale(K[i * n + k], VY[i * n + k])
                                     : c_scale(-K[i * n + k - n], VX[i * n + k - n]);
                    },
                    [=](int k, int j) { return k < n ? VX[k * n + j] : VY[(k - n) * n + j]; });
            wg_gemm_lds<false, false>(S, P, n, 2 * n,
                    [=](int i, int k) { return k < n ? VX[i * n + k] : VY[i * n + k - n]; },
                    [=](int k, int j) {
                        return k < n ? c_scale(-K[k * n + j], VY[k * n + j])
                                     : c_scale(K[(k - n) * n + j], VX[(k - n) * n + j]);
                    });
            for (int e = threadIdx.x; e < n * n; e += kWgThreads) {
                const int m = e / n, q = e - (e / n) * n;
                const double de = S.E[m] - S.E[q];
                HB[e] = (m != q && fabs(de) >= delta) ? c_scale(invN / de, c_i(c_add(W[e], P[e])))
                                                      : c_make(0.0, 0.0);
            }
            // the diagonal and the pairs closer than delta (neighbours in the sorted
            // spectrum): one wavefront per element, lanes over p
            {
                const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
                for (int m = wv; m < n; m += kWgThreads / 64) {
                    int qlo = m, qhi = m;
                    while (qlo > 0 && fabs(S.E[m] - S.E[qlo - 1]) < delta) --qlo;
                    while (qhi < n - 1 && fabs(S.E[qhi + 1] - S.E[m]) < delta) ++qhi;
                    for (int q = qlo; q <= qhi; ++q) {
                        const double xm = 0.5 * (S.E[m] + S.E[q]);
                        double phx, dphx;
                        if (m == q) {
                            phx = S.phi[m];
                            dphx = S.dphi[m];
                        } else {
                            wg_phi_at(xm, ef, sb, a.nF, a.kT, phx, dphx);
                        }
                        double2 acc = c_make(0.0, 0.0);
                        for (int p = lane; p < n; p += 64) {
                            const double x = xm - S.E[p];
                            const double den = x * x + eta2;
                            const double w = dphx / den - (phx - S.phi[p]) * 2.0 * x / (den * den);
                            double2 z = c_mul(B[m * n + p], A[p * n + q]);
                            z = c_fnma(A[m * n + p], B[p * n + q], z);
                            acc = c_add(acc, c_scale(w, z));
                        }
                        acc.x = wg_wave_reduce(acc.x, [](double x, double y) { return x + y; });
                        acc.y = wg_wave_reduce(acc.y, [](double x, double y) { return x + y; });
                        if (lane == 0) HB[m * n + q] = c_scale(invN, c_i(acc));
                    }
                }
            }
            __syncthreads();
            // Hbar = U Hbar' U^+  (P = Hbar' U^+, W = U P)
            wg_gemm<false, true>(S, P, n, [=](int i, int k) { return HB[i * n + k]; },
                    [=](int k, int j) { return c_conj(U[j * n + k]); });
            wg_gemm<false, false>(S, W, n, [=](int i, int k) { return U[i * n + k]; },
                    [=](int k, int j) { return P[k * n + j]; });
            // vbar_x = U Abar U^+, Abar = (i/N) K o B   (P = Abar U^+, VY = U P)
            wg_gemm<false, true>(S, P, n, [=](int i, int k) { return c_scale(invN * K[i * n + k], c_i(VY[i * n + k])); },
                    [=](int k, int j) { return c_conj(U[j * n + k]); });
            wg_gemm<false, false>(S, VY, n, [=](int i, int k) { return U[i * n + k]; },
                    [=](int k, int j) { return P[k * n + j]; });
            // vbar_y = U Bbar U^+, Bbar = -(i/N) K o A  (P = Bbar U^+, VX = U P)
            wg_gemm<false, true>(S, P, n, [=](int i, int k) { return c_scale(-invN * K[i * n + k], c_i(VX[i * n + k])); },
                    [=](int k, int j) { return c_conj(U[j * n + k]); });
            wg_gemm<false, false>(S, VX, n, [=](int i, int k) { return U[i * n + k]; },
                    [=](int k, int j) { return P[k * n + j]; });
            // the k-point's Hbar, vbar_x, vbar_y, whole, for the block's pencil sums (k_pacc)
            double2* Xk = reinterpret_cast<double2*>(a.xbuf) + it.xbuf_off + (long long)kk * 3 * nn;
            bool bad = false;
            for (int e = threadIdx.x; e < n * n; e += kWgThreads) {
                const double2 h = W[e], x = VY[e], y = VX[e];
                bad |= !isfinite(h.x + h.y + x.x + x.y + y.x + y.y);
                Xk[e] = h;
                Xk[nn + e] = x;
                Xk[2 * nn + e] = y;
            }
            if (bad) atomicOr(a.status, kStatNonFinite);
            __syncthreads();
        }
    }
}

static bool g_wg_attr = false;
static hipError_t wg_attrs() {
    if (g_wg_attr) return hipSuccess;
    const void* fns[] = {reinterpret_cast<const void*>(&k_forward_wg<true, false>),
                         reinterpret_cast<const void*>(&k_forward_wg<false, false>),
                         reinterpret_cast<const void*>(&k_forward_wg<true, true>),
                         reinterpret_cast<const void*>(&k_forward_wg<false, true>),
                         reinterpret_cast<const void*>(&k_adjoint_wg<true>),
                         reinterpret_cast<const void*>(&k_adjoint_wg<false>)};
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kWgBigLds);
        if (e != hipSuccess) return e;
    }
    g_wg_attr = true;
    return hipSuccess;
}

long long wg_slot_elems(int nmax) { return 7LL * nmax * nmax; }

hipError_t launch_forward_wg(const WgLaunch& L, int np, hipStream_t s) {
    if (L.item_count <= 0) return hipSuccess;
    if (!L.queue) return hipErrorInvalidValue;
    hipError_t e = wg_attrs();
    if (e != hipSuccess) return e;
    const int grid = L.item_count < L.max_groups ? L.item_count : L.max_groups;
    if (np <= 64) {
        if (L.tensor)
            hipLaunchKernelGGL((k_forward_wg<true, true>), dim3(grid), dim3(kWgThreads), kWgSmallLds, s, L);
        else
            hipLaunchKernelGGL((k_forward_wg<true, false>), dim3(grid), dim3(kWgThreads), kWgSmallLds, s, L);
    } else {
        if (L.tensor)
            hipLaunchKernelGGL((k_forward_wg<false, true>), dim3(grid), dim3(kWgThreads), kWgBigLds, s, L);
        else
            hipLaunchKernelGGL((k_forward_wg<false, false>), dim3(grid), dim3(kWgThreads), kWgBigLds, s, L);
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_wg(const WgLaunch& L, int np, hipStream_t s) {
    if (L.item_count <= 0) return hipSuccess;
    if (!L.queue || L.unit_k < 1 || L.unit_parts < 1) return hipErrorInvalidValue;
    hipError_t e = wg_attrs();
    if (e != hipSuccess) return e;
    const int units = L.item_count * L.unit_parts;
    const int grid = units < L.max_groups ? units : L.max_groups;
    if (np <= 64)
        hipLaunchKernelGGL(k_adjoint_wg<true>, dim3(grid), dim3(kWgThreads), kWgSmallLds, s, L);
    else
        hipLaunchKernelGGL(k_adjoint_wg<false>, dim3(grid), dim3(kWgThreads), kWgBigLds, s, L);
    return hipGetLastError();
}

}  // namespace kubo
