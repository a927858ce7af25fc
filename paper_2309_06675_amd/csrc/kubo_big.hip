// kubo_big.hip -- the large-n path (128 < n <= 512): the paper's matrix-parallel
// regime for large N_d (end of its section on the vectorised implementation),
// where one k-point's matrices are large enough to spread over many workgroups.
//
// A batch of k-points of one model (one k-point per work item) goes through a
// pipeline of kernels, each over the whole batch; per k-point the matrices live
// in a slice of the workspace (row-major, complex):
//   k_big_build    H, v_x, v_y from the pencil partial sums (many workgroups per k)
//   k_big_tridiag  Householder reduction to real tridiagonal T (one 1024-thread
//                  workgroup per k; the lower triangle of the trailing matrix in the
//                  slice, one pass over it per step)
//   k_big_eig      T split into unreduced blocks where an off-diagonal is negligible,
//                  then every eigenvalue by Sturm bisection within its block (a thread each)
//   k_big_vec      eigenvectors of T: a twisted factorisation per isolated eigenvalue,
//                  inverse iteration with reorthogonalisation for clustered ones
//   k_big_tfac     T factors of the compact WY form of 32 Householder reflectors
//   k_big_gemm     batched complex products on FP64 MFMA (64 x 64 tiles, many
//                  workgroups per k): the back-transformation U = Q Z block by block
//                  (W = V^+ Z, W' = T W, Z -= V W') and the rotations U^+ v U
//   k_big_curv     band-pair curvature and the Fermi sums into the item's slot
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kubo_cplx.h"
#include "kubo_internal.h"
#include "kubo_launch.h"

namespace kubo {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// the k-point slice of item b of a launch
struct BigSlice {
    double2 *H, *VX, *VY, *U, *X, *V, *W, *W2, *TF;
    double *d, *e, *E, *piv;
    double2* tau;
    int* blk;  // per eigenvalue: block start (low 16 bits) and size (high 16 bits)
};

__device__ __forceinline__ BigSlice big_slice(const BigLaunch& a, int b) {
    const BigLayout L = big_layout(a.n);
    double2* base = reinterpret_cast<double2*>(a.scratch) + (long long)b * a.per_k;
    double* dbl = reinterpret_cast<double*>(base);
    BigSlice s;
    s.H = base + L.H;
    s.VX = base + L.VX;
    s.VY = base + L.VY;
    s.U = base + L.U;
    s.X = base + L.X;
    s.V = base + L.V;
    s.W = base + L.W;    // kBigB x n
    s.W2 = base + L.W2;  // kBigB x n
    s.TF = base + L.TF;  // blocks x kBigB x kBigB
    s.tau = base + L.tau;
    s.d = dbl + L.d;
    s.e = dbl + L.e;
    s.E = dbl + L.E;
    s.piv = dbl + L.piv;  // 6 n doubles per eigenvalue thread
    s.blk = reinterpret_cast<int*>(dbl + L.blk);
    return s;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

}  // namespace

// ---------------------------------------------------------------------------
// step 1: H, v_x, v_y of item b (grid: (element tiles, items))
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_big_build(BigLaunch a) {
    __shared__ double2 ph[16];
    const int b = blockIdx.y;
    const BlockItem it = a.tb.blocks[a.item_begin + b];
    const ModelDev md = a.tb.models[it.model];
    const int n = a.n;
    const long long nn = (long long)n * n;
    const int* r0 = a.tb.r0val + md.r0_first;
    if (threadIdx.x < md.nR0) ph[threadIdx.x] = unit_phase((long long)it.i0 * r0[threadIdx.x], md.N0);
    __syncthreads();
    const BigSlice s = big_slice(a, b);
    const double2* T0 = reinterpret_cast<const double2*>(a.tbuf) + it.tbuf_off;
    const double2* T1 = T0 + (long long)md.nR0 * nn;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
         e += (long long)gridDim.x * blockDim.x) {
        double2 h = c_make(0.0, 0.0), x = c_make(0.0, 0.0), y = c_make(0.0, 0.0);
        for (int rho = 0; rho < md.nR0; ++rho) {
            const double2 t0 = T0[rho * nn + e], t1 = T1[rho * nn + e];
            h = c_fma(t0, ph[rho], h);
            x = c_fma(t0, c_scale((double)r0[rho], c_i(ph[rho])), x);
            y = c_fma(t1, ph[rho], y);
        }
        s.H[e] = h;
        s.VX[e] = x;
        s.VY[e] = y;
        s.V[e] = c_make(0.0, 0.0);
    }
}

// ---------------------------------------------------------------------------
// step 2a: Householder reduction of H (Hermitian, full storage on entry) to real
// tridiagonal T = Q^+ H Q, Q = H_0 ... H_{n-2}, H_k = I - tau_k v_k v_k^+ with
// v_k[k+1] = 1.  The reflectors go to V (column k, zero elsewhere), tau to tau,
// the diagonal to d and the off-diagonal to e.  One workgroup per k-point.
// The reduction is bound by the traffic of the trailing matrix, so (i) step k's
// rank-2 update and step k+1's product p = A v share one pass over it: column
// k+1 of the updated matrix is formed first (from the old values and step k's
// v, w), giving v_{k+1}; then the rest is updated, written back and accumulated
// into p_{k+1}; and (ii) after step 0 only the lower triangle (diagonal
// included) is read and written, each element serving both halves of the
// Hermitian product: A_ji (j > i) adds A_ji v_i to p_j (the row part) and
// conj(A_ji) v_j to p_i (the column part).  Wavefront w owns the rows j = w mod
// 16 of the triangle, lanes over 64-column segments of a row: its row parts are
// summed across the lanes (complete, as the row is its own), its column parts
// stay in registers per segment and are combined across the 16 wavefronts in a
// fixed order, so the result does not depend on scheduling.
// ---------------------------------------------------------------------------
namespace {

// reflector of x (m entries, x[0] the first) into v (v[0] = 1); returns tau and
// writes beta (the new subdiagonal entry); thread 0 decides, all threads scale.
__device__ __forceinline__ double2 big_reflector(double2* v, int m, double xn2, double& beta,
                                                 double2* sh, double* shb) {
    if (threadIdx.x == 0) {
        const double2 alpha = v[0];
        double bt;
        double2 tau, scal;
        if (xn2 == 0.0 && alpha.y == 0.0) {
            bt = alpha.x;
            tau = c_make(0.0, 0.0);
            scal = c_make(0.0, 0.0);
        } else {
            const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2);
            bt = -copysign(nrm, alpha.x);
            tau = c_make((bt - alpha.x) / bt, -alpha.y / bt);
            const double ar = alpha.x - bt, ai = alpha.y;
            const double den = 1.0 / (ar * ar + ai * ai);
            scal = c_make(ar * den, -ai * den);
        }
        sh[0] = tau;
        sh[1] = scal;
        *shb = bt;
    }
    __syncthreads();
    const double2 scal = sh[1];
    for (int i = threadIdx.x; i < m; i += blockDim.x)
        if (i > 0) v[i] = c_mul(v[i], scal);
    if (threadIdx.x == 0) v[0] = c_make(1.0, 0.0);
    beta = *shb;
    const double2 tau = sh[0];
    __syncthreads();
    return tau;
}

}  // namespace

// Sums q[0..3] (two complex numbers) over the 64 lanes by recursive halving:
// lanes 0, 16, 32, 48 end with the sums of q[0], q[1], q[2], q[3].
__device__ __forceinline__ double big_lane_sum4(double q0, double q1, double q2, double q3) {
    const int l = threadIdx.x & 63;
    const bool hi32 = (l & 32) != 0, hi16 = (l & 16) != 0;
    // offset 32: the lower half keeps q0, q1, the upper half q2, q3
    const double s0 = hi32 ? q0 : q2, s1 = hi32 ? q1 : q3;
    double k0 = hi32 ? q2 : q0, k1 = hi32 ? q3 : q1;
    k0 += __shfl_xor(s0, 32, 64);
    k1 += __shfl_xor(s1, 32, 64);
    // offset 16: keep one of the two
    double r = hi16 ? k1 : k0;
    r += __shfl_xor(hi16 ? k0 : k1, 16, 64);
    for (int off = 8; off >= 1; off >>= 1) r += __shfl_xor(r, off, 64);
    return r;
}

// NS: 64-column segments a row of the trailing triangle can span; RB: rows a
// wavefront takes at a time (their loads in flight together)
template <int NS, int RB>
__global__ __launch_bounds__(1024) void k_big_tridiag(BigLaunch a) {
    __shared__ double2 vb[2][kBigMaxN], w[kBigMaxN], p[kBigMaxN], cb[8][kBigMaxN];
    __shared__ double red[16];
    __shared__ double2 sh[2];
    __shared__ double shb;
    const int b = blockIdx.x;
    const int n = a.n;
    const BigSlice s = big_slice(a, b);
    double2* A = s.H;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int q4 = tid >> 8, c0 = tid & 255;  // step 0: four threads per column
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    double2 tau_cur;  // tau of the current step, in every thread
    double2(*pp)[kBigMaxN] = cb;
    // step 0: reflector of column 0 and p_0 = A v_0 (a plain pass)
    {
        const int m = n - 1;
        double2* v = vb[0];
        double xn2 = 0.0;
        for (int i = tid; i < m; i += nt) {
            const double2 x = A[(long long)(1 + i) * n];
            v[i] = x;
            if (i > 0) xn2 += x.x * x.x + x.y * x.y;
        }
        xn2 = block_sum(xn2, red);
        double beta;
        const double2 tau = big_reflector(v, m, xn2, beta, sh, &shb);
        tau_cur = tau;
        if (tid == 0) {
            s.d[0] = A[0].x;
            s.e[0] = beta;
            s.tau[0] = tau;
        }
        for (int i = tid; i < m; i += nt) s.V[(long long)(1 + i) * n] = v[i];
        for (int i = c0; i < m; i += 256) {
            double2 acc = c_make(0.0, 0.0);
            for (int j = q4; j < m; j += 4) acc = c_fmac(A[(long long)(1 + j) * n + 1 + i], v[j], acc);
            pp[q4][i] = acc;
        }
        __syncthreads();
        for (int i = tid; i < m; i += nt) p[i] = c_add(c_add(pp[0][i], pp[1][i]), c_add(pp[2][i], pp[3][i]));
        __syncthreads();
    }
    for (int k = 0; k < n - 1; ++k) {
        const int m = n - k - 1;  // step k works on rows and columns k+1 .. n-1
        double2* v = vb[k & 1];
        double2* vn = vb[(k + 1) & 1];
        const double2 tau = tau_cur;
        // w = tau p - (|tau|^2 (v^+ p) / 2) v (zero when tau = 0: then nothing changes)
        double mu = 0.0;
        for (int i = tid; i < m; i += nt) mu += v[i].x * p[i].x + v[i].y * p[i].y;
        mu = block_sum(mu, red);
        const double t2 = 0.5 * (tau.x * tau.x + tau.y * tau.y) * mu;
        for (int i = tid; i < m; i += nt) w[i] = c_sub(c_mul(tau, p[i]), c_scale(t2, v[i]));
        __syncthreads();
        if (m == 1) {  // the last diagonal entry
            if (tid == 0) {
                const double2 a11 = c_rank2c(A[(long long)(n - 1) * n + n - 1], v[0], w[0], w[0], v[0]);
                s.d[n - 1] = a11.x;
                s.e[n - 1] = 0.0;
                s.tau[n - 1] = c_make(0.0, 0.0);
            }
            break;
        }
        // column k+1 of the updated matrix below its diagonal (rows k+2 ..): x_i, and
        // the diagonal entry d_{k+1}
        const int mn = m - 1;
        double xn2 = 0.0;
        for (int i = tid; i < mn; i += nt) {
            const double2 x = c_rank2c(A[(long long)(k + 2 + i) * n + k + 1], v[1 + i], w[0], w[1 + i], v[0]);
            vn[i] = x;
            if (i > 0) xn2 += x.x * x.x + x.y * x.y;
        }
        xn2 = block_sum(xn2, red);
        double beta;
        const double2 taun = big_reflector(vn, mn, xn2, beta, sh, &shb);
        tau_cur = taun;
        if (tid == 0) {
            s.d[k + 1] = c_rank2c(A[(long long)(k + 1) * n + k + 1], v[0], w[0], w[0], v[0]).x;
            s.e[k + 1] = beta;
            s.tau[k + 1] = taun;
        }
        for (int i = tid; i < mn; i += nt) s.V[(long long)(k + 2 + i) * n + k + 1] = vn[i];
        // one pass over the lower triangle of rows/columns k+2.. (local x = global -
        // k - 2): A <- A - v w^+ - w v^+, and p_{k+1} = A' vn.  Column k+1 is done
        // (it gave vn), so it is neither updated nor stored.
        double2* const A0 = A + (long long)(k + 2) * n + (k + 2);
        const double2* const v1 = v + 1;
        const double2* const w1 = w + 1;
        double2 pc[NS];
#pragma unroll
        for (int sg = 0; sg < NS; ++sg) pc[sg] = c_make(0.0, 0.0);
        for (int j0 = wv; j0 < mn; j0 += 16 * RB) {
            double2 av[RB][NS];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int jx = j0 + 16 * r;
#pragma unroll
                for (int sg = 0; sg < NS; ++sg) {
                    const int ix = 64 * sg + lane;
                    av[r][sg] = c_make(0.0, 0.0);
                    if (jx < mn && ix <= jx) av[r][sg] = A0[(long long)jx * n + ix];
                }
            }
            double rs[RB][2];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int jx = j0 + 16 * r;
                double2 acc = c_make(0.0, 0.0);
                if (jx < mn) {
                    const double2 vj = v1[jx], wj = w1[jx], vnj = vn[jx];
#pragma unroll
                    for (int sg = 0; sg < NS; ++sg) {
                        const int ix = 64 * sg + lane;
                        if (ix <= jx) {
                            const double2 na = c_rank2c(av[r][sg], vj, w1[ix], wj, v1[ix]);
                            A0[(long long)jx * n + ix] = na;
                            pc[sg] = c_fmac(na, vnj, pc[sg]);
                            if (ix < jx) acc = c_fma(na, vn[ix], acc);
                        }
                    }
                }
                rs[r][0] = acc.x;
                rs[r][1] = acc.y;
            }
            // the row parts: lanes 0/16 (and 32/48) end with row j0's (j0 + 16's) sum
#pragma unroll
            for (int r = 0; r < RB; r += 2) {
                const double q2 = (r + 1 < RB) ? rs[r + 1][0] : 0.0;
                const double q3 = (r + 1 < RB) ? rs[r + 1][1] : 0.0;
                const double sum = big_lane_sum4(rs[r][0], rs[r][1], q2, q3);
                const int jx = j0 + 16 * (r + (lane >> 5));
                if ((lane & 15) == 0 && jx < mn && (r + (lane >> 5)) < RB)
                    reinterpret_cast<double*>(p)[2 * jx + ((lane >> 4) & 1)] = sum;
            }
        }
        // the column parts: wavefronts 8..15 hand theirs to 0..7, which add their own
        if (wv >= 8) {
#pragma unroll
            for (int sg = 0; sg < NS; ++sg) {
                const int ix = 64 * sg + lane;
                if (ix < mn) cb[wv - 8][ix] = pc[sg];
            }
        }
        __syncthreads();
        if (wv < 8) {
#pragma unroll
            for (int sg = 0; sg < NS; ++sg) {
                const int ix = 64 * sg + lane;
                if (ix < mn) cb[wv][ix] = c_add(cb[wv][ix], pc[sg]);
            }
        }
        __syncthreads();
        for (int i = tid; i < mn; i += nt) {
            double2 t = p[i];
#pragma unroll
            for (int u = 0; u < 8; ++u) t = c_add(t, cb[u][i]);
            p[i] = t;
        }
        __syncthreads();
    }
    if (n == 1 && tid == 0) {
        s.d[0] = A[0].x;
        s.e[0] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// step 2b: eigenvalues.  T splits where |e_i| <= eps (|d_i| + |d_i+1|); within an
// unreduced block every eigenvalue is simple, found from Sturm counts on the block
// (ratio form with a pivot floor, d and e staged in LDS) to 4 eps max|lambda|: by
// trisection with two lanes per eigenvalue when 2n threads fit the block, else by
// bisection.  The j-th eigenvalue in block order goes to thread (pair) j
// (eigenvalues are not sorted: nothing downstream needs an order).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBigMaxN) void k_big_eig(BigLaunch a) {
    __shared__ int bstart[kBigMaxN], bsize[kBigMaxN], boff[kBigMaxN];
    __shared__ double dd[kBigMaxN], ee[kBigMaxN];
    __shared__ int nblk;
    __shared__ double sh_lo, sh_hi, sh_emax;
    const int b = blockIdx.x;
    const int n = a.n;
    const BigSlice s = big_slice(a, b);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        dd[i] = s.d[i];
        ee[i] = s.e[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double lo = 1e300, hi = -1e300, emax = 0.0;
        int nb = 0, start = 0;
        for (int i = 0; i < n; ++i) {
            const double ep = (i > 0) ? fabs(ee[i - 1]) : 0.0, en = (i < n - 1) ? fabs(ee[i]) : 0.0;
            lo = fmin(lo, dd[i] - ep - en);
            hi = fmax(hi, dd[i] + ep + en);
            emax = fmax(emax, en);
            const bool cut = (i == n - 1) || en <= 2.220446049250313e-16 * (fabs(dd[i]) + fabs(dd[i + 1]));
            if (cut) {
                bstart[nb] = start;
                bsize[nb] = i + 1 - start;
                boff[nb] = start;
                ++nb;
                start = i + 1;
            }
        }
        nblk = nb;
        sh_lo = lo;
        sh_hi = hi;
        sh_emax = emax;
    }
    __syncthreads();
    // two lanes of a wavefront per eigenvalue when the block has the threads for it:
    // each pass they count at the two points that cut the interval in thirds and
    // keep the third holding the eigenvalue; otherwise one thread bisects
    const bool pair = 2 * n <= (int)blockDim.x;
    const int j = pair ? (threadIdx.x >> 1) : threadIdx.x;
    const int half = pair ? (threadIdx.x & 1) : 0;
    if (j >= n) return;  // whole pairs leave together
    int bi = 0;
    while (bi + 1 < nblk && boff[bi + 1] <= j) ++bi;
    const int st = bstart[bi], m = bsize[bi], jl = j - st;
    const double scale = fmax(fabs(sh_lo), fabs(sh_hi));
    const double tol = 4.0 * 2.220446049250313e-16 * scale + 1e-300;
    const double pivmin = 1e-290 * fmax(1.0, sh_emax * sh_emax);
    // eigenvalues of the block below x (Sturm count of the ratio recurrence)
    auto count = [&](double x) {
        int cnt = 0;
        double q = 1.0;
        for (int i = st; i < st + m; ++i) {
            const double e2 = (i > st) ? ee[i - 1] * ee[i - 1] : 0.0;
            double r = __builtin_amdgcn_rcp(q);
            r = fma(r, fma(-q, r, 1.0), r);
            double qi = fma(-e2, r, dd[i] - x);
            if (fabs(qi) < pivmin) qi = -pivmin;
            cnt += (qi < 0.0) ? 1 : 0;
            q = qi;
        }
        return cnt;
    };
    double lo = sh_lo, hi = sh_hi;
    bool ok = false;
    for (int pass = 0; pass < 200; ++pass) {
        if (hi - lo <= tol) {
            ok = true;
            break;
        }
        if (pair) {
            const double t = (hi - lo) * (1.0 / 3.0);
            const double x1 = lo + t, x2 = hi - t;  // the same in both lanes
            const int c = count(half ? x2 : x1);
            const int co = __shfl_xor(c, 1);
            const int c1 = half ? co : c, c2 = half ? c : co;
            if (c1 > jl) {
                hi = x1;
            } else if (c2 > jl) {
                lo = x1;
                hi = x2;
            } else {
                lo = x2;
            }
        } else {
            const double x = 0.5 * (lo + hi);
            if (count(x) <= jl) lo = x;
            else hi = x;
        }
    }
    if (half == 0) {
        s.E[j] = 0.5 * (lo + hi);
        s.blk[j] = st | (m << 16);
        if (!ok) atomicOr(a.status, kStatNoConv);
    }
}

// ---------------------------------------------------------------------------
// step 2c: eigenvectors of T into Z (stored in U, real, column j, zero outside
// the block).  An eigenvalue whose relative gap to its block neighbours is at
// least kBigGap takes one twisted factorisation (error eps |T| / gap); a cluster
// is solved by its first member's thread, member by member, with inverse
// iteration from a fixed pseudo-random start (splitmix64 of the index) and
// modified Gram-Schmidt against the cluster's earlier members after each solve.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double big_start(int j, int i) {
    unsigned long long z = 0x9E3779B97F4A7C15ull * (unsigned long long)(j * 1315423911u + i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

// solve (T - lam I) y = x on rows [st, st+m) by Gaussian elimination with partial
// pivoting (the tridiagonal LU keeps a second superdiagonal); y overwrites x.
// u0, u1, u2, l: scratch of m doubles each.
__device__ void big_tri_solve(const double* d, const double* e, int st, int m, double lam,
                              double pivmin, double* x, double* u0, double* u1, double* u2,
                              double* l, int* pv) {
    // rows i: diag d_i - lam, sub/super e_i
    double a0 = d[st] - lam, a1 = (m > 1) ? e[st] : 0.0, a2 = 0.0;
    for (int i = 0; i < m - 1; ++i) {
        const double sub = e[st + i];
        const double b0 = d[st + i + 1] - lam, b1 = (i + 1 < m - 1) ? e[st + i + 1] : 0.0;
        if (fabs(sub) > fabs(a0)) {  // swap rows i and i+1
            pv[i] = 1;
            u0[i] = sub;
            u1[i] = b0;
            u2[i] = b1;
            const double f = a0 / sub;
            l[i] = f;
            a0 = a1 - f * b0;
            a1 = a2 - f * b1;
            a2 = 0.0;
        } else {
            pv[i] = 0;
            if (fabs(a0) < pivmin) a0 = pivmin;
            u0[i] = a0;
            u1[i] = a1;
            u2[i] = a2;
            const double f = sub / a0;
            l[i] = f;
            a0 = b0 - f * a1;
            a1 = b1;
            a2 = 0.0;
        }
    }
    if (fabs(a0) < pivmin) a0 = pivmin;
    u0[m - 1] = a0;
    u1[m - 1] = 0.0;
    u2[m - 1] = 0.0;
    // forward: apply the row swaps and multipliers to x
    for (int i = 0; i < m - 1; ++i) {
        if (pv[i]) {
            const double t = x[i];
            x[i] = x[i + 1];
            x[i + 1] = t - l[i] * x[i];
        } else {
            x[i + 1] -= l[i] * x[i];
        }
    }
    // back substitution with the upper factor (bandwidth 3)
    for (int i = m - 1; i >= 0; --i) {
        double r = x[i];
        if (i + 1 < m) r -= u1[i] * x[i + 1];
        if (i + 2 < m) r -= u2[i] * x[i + 2];
        x[i] = r / u0[i];
    }
}

__global__ __launch_bounds__(kBigMaxN) void k_big_vec(BigLaunch a) {
    __shared__ double dd[kBigMaxN], ee[kBigMaxN];  // T, read by every thread's recurrences
    const int b = blockIdx.x;
    const int n = a.n;
    const BigSlice s = big_slice(a, b);
    const int j = threadIdx.x;
    for (long long e = j; e < (long long)n * n; e += blockDim.x) s.U[e] = c_make(0.0, 0.0);
    for (int i = j; i < n; i += blockDim.x) {
        dd[i] = s.d[i];
        ee[i] = s.e[i];
    }
    __syncthreads();
    if (j >= n) return;
    const int st = s.blk[j] & 0xffff, m = s.blk[j] >> 16;
    const double lam = s.E[j];
    double span = 0.0, emax = 0.0;
    for (int i = st; i < st + m; ++i) {
        span = fmax(span, fabs(dd[i]) + ((i > st) ? fabs(ee[i - 1]) : 0.0) + ((i < st + m - 1) ? fabs(ee[i]) : 0.0));
        emax = fmax(emax, (i < st + m - 1) ? fabs(ee[i]) : 0.0);
    }
    const double pivmin = 1e-290 * fmax(1.0, emax * emax);
    const double gapmin = kBigGap * fmax(span, 1e-300);
    // neighbours in the same block (eigenvalues of a block are consecutive in j)
    auto close = [&](int q) { return q >= st && q < st + m && fabs(s.E[q] - lam) < gapmin; };
    const bool clustered = close(j - 1) || close(j + 1);
    double* dp = s.piv + (long long)j * 6 * n;  // this thread's six rows of n
    double* dm = dp + n;
    if (!clustered) {
        // twisted factorisation of T - lam I on the block
        double q = 1.0;
        for (int i = 0; i < m; ++i) {
            double qi = (dd[st + i] - lam) - ((i > 0) ? ee[st + i - 1] * ee[st + i - 1] / q : 0.0);
            if (fabs(qi) < pivmin) qi = -pivmin;
            dp[i] = qi;
            q = qi;
        }
        q = 1.0;
        for (int i = m - 1; i >= 0; --i) {
            double qi = (dd[st + i] - lam) - ((i < m - 1) ? ee[st + i] * ee[st + i] / q : 0.0);
            if (fabs(qi) < pivmin) qi = -pivmin;
            dm[i] = qi;
            q = qi;
        }
        int r = 0;
        double best = 1e300;
        for (int i = 0; i < m; ++i) {
            const double g = dp[i] + dm[i] - (dd[st + i] - lam);
            if (fabs(g) < best) {
                best = fabs(g);
                r = i;
            }
        }
        // z_r = 1; z_i = -e_i z_{i+1} / dp_i (i < r); z_i = -e_{i-1} z_{i-1} / dm_i (i > r)
        double nrm = 1.0;
        dp[r] = 1.0;  // dp reused for z
        for (int i = r - 1; i >= 0; --i) {
            const double z = -ee[st + i] * dp[i + 1] / dp[i];
            dp[i] = z;
            nrm += z * z;
        }
        double zp = 1.0;
        for (int i = r + 1; i < m; ++i) {
            const double z = -ee[st + i - 1] * zp / dm[i];
            dm[i] = z;
            zp = z;
            nrm += z * z;
        }
        const double inv = 1.0 / sqrt(nrm);
        for (int i = 0; i < m; ++i) {
            const double z = (i <= r) ? dp[i] : dm[i];
            s.U[(long long)(st + i) * n + j] = c_make(z * inv, 0.0);
        }
        if (!isfinite(inv)) atomicOr(a.status, kStatNonFinite);
        return;
    }
    // a cluster (a run of eigenvalues of one block with consecutive gaps below
    // gapmin): its first member does all of it, in its own six rows
    if (close(j - 1)) return;
    int last = j;
    while (last + 1 < st + m && s.E[last + 1] - s.E[last] < gapmin) ++last;
    double* x = dp;
    double* u0 = dm;
    double* u1 = dp + 2 * n;
    double* u2 = dp + 3 * n;
    double* l = dp + 4 * n;
    int* pv = reinterpret_cast<int*>(dp + 5 * n);
    const double floor_solve = 2.220446049250313e-16 * fmax(span, 1e-300);
    for (int c = j; c <= last; ++c) {
        const double lc = s.E[c] + (double)(c - j) * 2.220446049250313e-16 * span;  // separate the shifts
        for (int i = 0; i < m; ++i) x[i] = big_start(c, i);
        for (int itr = 0; itr < 3; ++itr) {
            big_tri_solve(dd, ee, st, m, lc, floor_solve, x, u0, u1, u2, l, pv);
            // orthogonalise against the cluster's earlier members (modified Gram-Schmidt)
            for (int c2 = j; c2 < c; ++c2) {
                double dot = 0.0;
                for (int i = 0; i < m; ++i) dot += s.U[(long long)(st + i) * n + c2].x * x[i];
                for (int i = 0; i < m; ++i) x[i] -= dot * s.U[(long long)(st + i) * n + c2].x;
            }
            double nrm = 0.0;
            for (int i = 0; i < m; ++i) nrm += x[i] * x[i];
            const double inv = 1.0 / sqrt(nrm);
            for (int i = 0; i < m; ++i) x[i] *= inv;
        }
        for (int i = 0; i < m; ++i) s.U[(long long)(st + i) * n + c] = c_make(x[i], 0.0);
    }
}

// ---------------------------------------------------------------------------
// step 2d: T factors of the reflector blocks (kBigB reflectors per block,
// columns k0 .. k0+kBigB-1 of V): TF = upper triangular with TF_jj = tau_j,
// TF(0:j, j) = -tau_j TF(0:j, 0:j) (V(:, 0:j)^+ v_j)  (compact WY, Schreiber and
// Van Loan 1989).  grid: (blocks, items), 256 threads.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_big_tfac(BigLaunch a) {
    __shared__ double2 C[kBigB][kBigB + 1];
    __shared__ double2 T[kBigB][kBigB + 1];
    const int blk = blockIdx.x, b = blockIdx.y;
    const int n = a.n;
    const BigSlice s = big_slice(a, b);
    const int k0 = blk * kBigB;
    const int bs = min(kBigB, n - 1 - k0);
    for (int e = threadIdx.x; e < kBigB * kBigB; e += blockDim.x) {
        const int i = e / kBigB, j = e - (e / kBigB) * kBigB;
        double2 acc = c_make(0.0, 0.0);
        if (i < j && j < bs) {
            // four rows at a time into four sums, so that eight loads are in flight
            const double2* vi = s.V + k0 + i;
            const double2* vj = s.V + k0 + j;
            double2 a4[4] = {acc, acc, acc, acc};
            int r = k0 + j + 1;
            for (; r + 3 < n; r += 4) {
                double2 x[4], y[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    x[u] = vi[(long long)(r + u) * n];
                    y[u] = vj[(long long)(r + u) * n];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) a4[u] = c_fmac(x[u], y[u], a4[u]);
            }
            for (; r < n; ++r) a4[0] = c_fmac(vi[(long long)r * n], vj[(long long)r * n], a4[0]);
            acc = c_add(c_add(a4[0], a4[1]), c_add(a4[2], a4[3]));
        }
        C[i][j] = acc;
        T[i][j] = c_make(0.0, 0.0);
    }
    __syncthreads();
    for (int j = 0; j < bs; ++j) {
        const double2 tj = s.tau[k0 + j];
        const int i = threadIdx.x;
        if (i < j) {
            double2 acc = c_make(0.0, 0.0);
            for (int l = i; l < j; ++l) acc = c_fma(T[i][l], C[l][j], acc);
            T[i][j] = c_mul(c_make(-tj.x, -tj.y), acc);
        } else if (i == j) {
            T[j][j] = tj;
        }
        __syncthreads();
    }
    double2* out = s.TF + (long long)blk * kBigB * kBigB;
    for (int e = threadIdx.x; e < kBigB * kBigB; e += blockDim.x) out[e] = T[e / kBigB][e % kBigB];
}

// ---------------------------------------------------------------------------
// batched complex product C = alpha op(A) op(B) + beta C (alpha = +-1, beta = 0 or 1)
// on FP64 MFMA: one 64 x 64 tile of C per 256-thread workgroup (grid: (N tiles,
// M tiles, items)), panels of 16 inner indices staged through LDS with coalesced
// reads, each wavefront a 32 x 32 block as 2 x 2 tiles of v_mfma_f64_16x16x4 (four
// real products per complex one).  op: 0 = as stored (row-major, leading dimension
// ld), 1 = conjugate transpose.  The operands are addressed as base + item * stride.
// ---------------------------------------------------------------------------
template <int OPA, int OPB>
__global__ __launch_bounds__(256) void k_big_gemm(BigGemm g) {
    constexpr int KT = 16, LDA = KT + 1, LDB = 64 + 1;
    __shared__ double2 As[64 * LDA];
    __shared__ double2 Bs[KT * LDB];
    const int b = blockIdx.z;
    const double2* A = g.A + (long long)b * g.sa;
    const double2* B = g.B + (long long)b * g.sb;
    double2* C = g.C + (long long)b * g.sc;
    const int i0 = 64 * blockIdx.y, j0 = 64 * blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int gq = lane >> 4, c = lane & 15, wr = w >> 1, wc = w & 1;
    const v4d zero = {0.0, 0.0, 0.0, 0.0};
    v4d cr[2][2], ci[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            cr[x][y] = zero;
            ci[x][y] = zero;
        }
    // panel elements of this thread: loaded into registers one panel ahead (indices
    // clamped into the matrices, so every load is valid and none waits behind a
    // branch), stored to LDS with zeros outside the matrices
    constexpr int PER = 64 * KT / 256;
    double2 ra[PER], rb[PER];
    auto load_panel = [&](int kb) {
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int e = tid + 256 * r;
            {
                const int ii = OPA ? (e & 63) : (e / KT), kk = OPA ? (e >> 6) : (e - (e / KT) * KT);
                const int gi = min(i0 + ii, g.M - 1), gk = min(kb + kk, g.K - 1);
                ra[r] = OPA ? c_conj(A[gk * g.lda + gi]) : A[gi * g.lda + gk];
            }
            {
                const int jj = OPB ? (e / KT) : (e & 63), kk = OPB ? (e - (e / KT) * KT) : (e >> 6);
                const int gj = min(j0 + jj, g.N - 1), gk = min(kb + kk, g.K - 1);
                rb[r] = OPB ? c_conj(B[gj * g.ldb + gk]) : B[gk * g.ldb + gj];
            }
        }
    };
    load_panel(0);
    for (int kb = 0; kb < g.K; kb += KT) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int e = tid + 256 * r;
            {
                const int ii = OPA ? (e & 63) : (e / KT), kk = OPA ? (e >> 6) : (e - (e / KT) * KT);
                As[ii * LDA + kk] = (i0 + ii < g.M && kb + kk < g.K) ? ra[r] : c_make(0.0, 0.0);
            }
            {
                const int jj = OPB ? (e / KT) : (e & 63), kk = OPB ? (e - (e / KT) * KT) : (e >> 6);
                Bs[kk * LDB + jj] = (j0 + jj < g.N && kb + kk < g.K) ? rb[r] : c_make(0.0, 0.0);
            }
        }
        __syncthreads();
        if (kb + KT < g.K) load_panel(kb + KT);  // in flight during this panel's products
#pragma unroll
        for (int k4 = 0; k4 < KT / 4; ++k4) {
            double2 av[2], bv[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                av[t] = As[(32 * wr + 16 * t + c) * LDA + 4 * k4 + gq];
                bv[t] = Bs[(4 * k4 + gq) * LDB + 32 * wc + 16 * t + c];
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    cr[x][y] = mfma(av[x].x, bv[y].x, cr[x][y]);
                    ci[x][y] = mfma(av[x].x, bv[y].y, ci[x][y]);
                    cr[x][y] = mfma(-av[x].y, bv[y].y, cr[x][y]);
                    ci[x][y] = mfma(av[x].y, bv[y].x, ci[x][y]);
                }
        }
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = i0 + 32 * wr + 16 * x + gq + 4 * q, col = j0 + 32 * wc + 16 * y + c;
                if (row < g.M && col < g.N) {
                    double2& o = C[(long long)row * g.ldc + col];
                    const double2 v = c_make(g.alpha * cr[x][y][q], g.alpha * ci[x][y][q]);
                    o = g.beta ? c_add(o, v) : v;
                }
            }
}

// ---------------------------------------------------------------------------
// step 4: Omega_n = -2 sum_{m != n} Im(A_nm B_mn) g(E_n - E_m) (B_mn = conj(B_nm))
// from A in VX and B in VY, then sum_n f(E_n; E_F[j]) Omega_n into the item's slot.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBigMaxN) void k_big_curv(BigLaunch a) {
    __shared__ double Om[kBigMaxN], Ev[kBigMaxN];
    const int b = blockIdx.x;
    const BlockItem it = a.tb.blocks[a.item_begin + b];
    const ModelDev md = a.tb.models[it.model];
    const int n = a.n;
    const BigSlice s = big_slice(a, b);
    const double eta2 = a.eta * a.eta;
    const int t = threadIdx.x;
    if (t < n) {
        const double en = s.E[t];
        double om = 0.0;
        for (int m = 0; m < n; ++m) {
            if (m == t) continue;
            const double2 x = s.VX[(long long)t * n + m], y = s.VY[(long long)t * n + m];
            const double de = en - s.E[m];
            const double den = de * de + eta2;
            // Im(A_nm conj(B_nm))
            if (den > 0.0) om += (x.y * y.x - x.x * y.y) / den;
        }
        Om[t] = -2.0 * om;
        Ev[t] = en;
    }
    __syncthreads();
    double* part = a.partial + (long long)it.slot * a.nF;
    const double* ef = a.e_fermi + md.f_off;
    const double ikT = (a.kT > 0.0) ? 1.0 / a.kT : 0.0;
    for (int j = t; j < a.nF; j += blockDim.x) {
        double sum = 0.0;
        for (int m = 0; m < n; ++m) sum += occupation_ikt(Ev[m], ef[j], a.kT, ikT) * Om[m];
        if (!isfinite(sum)) atomicOr(a.status, kStatNonFinite);
        part[j] = sum;
    }
}

// ---------------------------------------------------------------------------
// host side: the pipeline for `count` items of one model of size n
// ---------------------------------------------------------------------------
static hipError_t gemm(int opa, int opb, const BigGemm& g, int items, hipStream_t s) {
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, items);
    if (opa == 0 && opb == 0) hipLaunchKernelGGL((k_big_gemm<0, 0>), grid, dim3(256), 0, s, g);
    else if (opa == 1 && opb == 0) hipLaunchKernelGGL((k_big_gemm<1, 0>), grid, dim3(256), 0, s, g);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_big_forward(const BigLaunch& L, hipStream_t s, hipEvent_t red_start, hipEvent_t red_stop) {
    if (L.count <= 0) return hipSuccess;
    if (L.n < 2 || L.n > kBigMaxN) return hipErrorInvalidValue;
    const int n = L.n;
    const long long nn = (long long)n * n;
    const long long pk = L.per_k;
    const BigLayout Y = big_layout(n);
    if (pk < Y.per_k) return hipErrorInvalidValue;
    hipError_t e;
    hipLaunchKernelGGL(k_big_build, dim3((unsigned)((nn + 255) / 256 < 64 ? (nn + 255) / 256 : 64), L.count),
                       dim3(256), 0, s, L);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (red_start && (e = hipEventRecord(red_start, s)) != hipSuccess) return e;
    if (L.n <= 258)
        hipLaunchKernelGGL((k_big_tridiag<4, 2>), dim3(L.count), dim3(1024), 0, s, L);
    else
        hipLaunchKernelGGL((k_big_tridiag<8, 1>), dim3(L.count), dim3(1024), 0, s, L);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (red_stop && (e = hipEventRecord(red_stop, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_big_eig, dim3(L.count), dim3(kBigMaxN), 0, s, L);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_big_vec, dim3(L.count), dim3(kBigMaxN), 0, s, L);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int nb = (n - 1 + kBigB - 1) / kBigB;  // reflector blocks (n - 1 reflectors)
    hipLaunchKernelGGL(k_big_tfac, dim3(nb, L.count), dim3(256), 0, s, L);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the matrices of the first slice (the products step by per_k from item to item)
    double2* base = reinterpret_cast<double2*>(L.scratch);
    double2* VX = base + Y.VX;
    double2* VY = base + Y.VY;
    double2* U = base + Y.U;
    double2* X = base + Y.X;
    double2* V = base + Y.V;
    double2* W = base + Y.W;
    double2* W2 = base + Y.W2;
    double2* TF = base + Y.TF;
    // back-transformation: Z (in U) <- Q_b Z for the blocks from last to first
    for (int blk = nb - 1; blk >= 0; --blk) {
        const int k0 = blk * kBigB;
        const int bs = (n - 1 - k0) < kBigB ? (n - 1 - k0) : kBigB;
        BigGemm g{};
        // the block's reflectors are zero above row k0 + 1: both products skip those rows
        const long long r1 = (long long)(k0 + 1) * n;
        const int mr = n - k0 - 1;
        // W = V_b^+ Z  (bs x n)
        g.A = V + r1 + k0; g.lda = n; g.sa = pk;
        g.B = U + r1; g.ldb = n; g.sb = pk;
        g.C = W; g.ldc = n; g.sc = pk;
        g.M = bs; g.N = n; g.K = mr; g.alpha = 1.0; g.beta = 0;
        if ((e = gemm(1, 0, g, L.count, s)) != hipSuccess) return e;
        // W2 = T W  (bs x n)
        g.A = TF + (long long)blk * kBigB * kBigB; g.lda = kBigB; g.sa = pk;
        g.B = W; g.ldb = n; g.sb = pk;
        g.C = W2; g.ldc = n; g.sc = pk;
        g.M = bs; g.N = n; g.K = bs; g.alpha = 1.0; g.beta = 0;
        if ((e = gemm(0, 0, g, L.count, s)) != hipSuccess) return e;
        // Z -= V_b W2  (rows k0 + 1 .. of Z)
        g.A = V + r1 + k0; g.lda = n; g.sa = pk;
        g.B = W2; g.ldb = n; g.sb = pk;
        g.C = U + r1; g.ldc = n; g.sc = pk;
        g.M = mr; g.N = n; g.K = bs; g.alpha = -1.0; g.beta = 1;
        if ((e = gemm(0, 0, g, L.count, s)) != hipSuccess) return e;
    }
    // rotations: X = v U, then v' = U^+ X into the velocity's own buffer
    for (double2* Vel : {VX, VY}) {
        BigGemm g{};
        g.A = Vel; g.lda = n; g.sa = pk;
        g.B = U; g.ldb = n; g.sb = pk;
        g.C = X; g.ldc = n; g.sc = pk;
        g.M = n; g.N = n; g.K = n; g.alpha = 1.0; g.beta = 0;
        if ((e = gemm(0, 0, g, L.count, s)) != hipSuccess) return e;
        g.A = U; g.lda = n; g.sa = pk;
        g.B = X; g.ldb = n; g.sb = pk;
        g.C = Vel; g.ldc = n; g.sc = pk;
        if ((e = gemm(1, 0, g, L.count, s)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_big_curv, dim3(L.count), dim3(kBigMaxN), 0, s, L);
    return hipGetLastError();
}

}  // namespace kubo
