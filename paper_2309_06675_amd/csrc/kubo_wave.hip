// kubo_wave.hip -- one wavefront per k-point: the forward pipeline for n <= 32
// and its adjoint.
//
// Eigensolver: the route the paper batched from EISPACK for complex Hermitian
// matrices (Householder reduction to a real symmetric tridiagonal matrix, the
// tridiagonal eigenproblem, back-transformation), restated for a 64-lane
// wavefront instead of one vector lane per matrix:
//   * Householder: the matrix stays in registers, lane pair (2i, 2i+1) holding
//     row i with the columns interleaved between the two lanes; the reflector of
//     column k is chosen so the sub-diagonal element is real, making T real.
//   * Eigenvalues: Sturm counts with safeguarded Newton steps, two lanes per
//     eigenvalue; eigenvectors of T: one twisted factorisation per lane pair.
//     Spectra with a relative gap below 1e-3 take implicit QL instead (the
//     tridiagonal one element per lane, the rotations applied to Z one row per
//     lane).
//   * Back-transformation U = H_0 ... H_{n-2} Z: lane pair per column, rows
//     interleaved between the two lanes.
// H, v_x and v_y are summed over their upper triangles (they are Hermitian) and
// mirrored.  Velocities (n > 8): A = U^+ v_x U and B = U^+ v_y U are dense
// complex products, done on the FP64 matrix cores (16x16x4 MFMA, four real
// products per complex one).  v is staged in LDS, U is read once per k-point
// into the MFMA operand layout and reused by both products of both
// velocities, and the first product's accumulators feed the second directly
// (X = v U, then M = X^+ U with the contraction index permuted so that every
// lane already holds its operand).  The curvature is taken from the
// accumulator tiles.  For n <= 8: W = v U with v built on the fly, U^+ W
// accumulated in registers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kubo_cplx.h"
#include "kubo_internal.h"
#include "kubo_launch.h"

namespace kubo {

// Cross-lane reductions without the LDS crossbar: DPP inside each row of 16
// lanes, then the gfx950 row-swap instructions across rows and halves.  Every
// lane ends with the same bits (each step combines the same two operands).
__device__ __forceinline__ double dpp_xor1(double v) {
    return __builtin_amdgcn_update_dpp(0.0, v, 0xB1, 0xF, 0xF, false);
}

__device__ __forceinline__ double join_u32(unsigned lo, unsigned hi) {
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <class Op>
__device__ __forceinline__ double wave_allreduce(double v, Op op) {
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));   // lane ^ 1
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));   // lane ^ 2
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false));  // 7 - lane within 8
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false));  // 15 - lane within 16
    {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
        v = op(join_u32(lo[0], hi[0]), join_u32(lo[1], hi[1]));  // rows (0, 1) and (2, 3)
    }
    {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
        v = op(join_u32(lo[0], hi[0]), join_u32(lo[1], hi[1]));  // the two halves
    }
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
    return wave_allreduce(v, [](double x, double y) { return x + y; });
}
__device__ __forceinline__ double wave_min(double v) {
    return wave_allreduce(v, [](double x, double y) { return fmin(x, y); });
}
__device__ __forceinline__ double wave_max(double v) {
    return wave_allreduce(v, [](double x, double y) { return fmax(x, y); });
}

// value of a per-lane register held by lane `src` (src must be wave-uniform)
__device__ __forceinline__ double lane_read(double v, int src) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), src);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

typedef double v4d __attribute__((ext_vector_type(4)));

// D = A B + C for a 16x4 (A) by 4x16 (B) FP64 tile.  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; D[l / 16 + 4 q][l % 16] is
// element q of lane l's accumulator.
__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// sum over the 16 lanes of a DPP row (lanes 16r .. 16r+15); every lane gets it
__device__ __forceinline__ double row16_sum(double v) {
    v += __builtin_amdgcn_update_dpp(0.0, v, 0xB1, 0xF, 0xF, false);   // lane ^ 1
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x4E, 0xF, 0xF, false);   // lane ^ 2
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x141, 0xF, 0xF, false);  // 7 - lane within 8
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x140, 0xF, 0xF, false);  // 15 - lane within 16
    return v;
}

template <int NP>
struct WaveLds {
    static constexpr int LD = NP + 1;
    double2 P[NP * LD];  // H, then the Householder vectors, then W = v U
    double2 U[NP * LD];  // Z (real parts) during QL, then U
    double2 tau[NP];
    double2 vv[NP];
    double2 wv[NP];
    double cs[2 * NP];
    double2 de2[NP];  // (d_i, e_i) of the tridiagonal matrix, zero past n
    double E[NP];
    double Om[NP];
    double phi[NP];   // adjoint: phi(E_b) = sum_j sbar_j f_j(E_b)
    double dphi[NP];  // and its derivative
    double2 ph[16];
};

// Reduce the Hermitian matrix in S.P (n x n) to real tridiagonal form.
// The matrix lives in registers: lane 2i + h holds row i, columns 2 jj + h
// (jj < NP/2).  Each step broadcasts the reflector v and the vector w through
// LDS and applies A <- A - v w^+ - w v^+ in registers; groups of four slots
// whose eight columns are all reduced already are skipped (a wave-uniform
// test), which saves about 40% of the work over the whole reduction.
// On return lane i holds d_i and e_i (e_{n-1} = 0); the Householder vector of
// step k is stored in S.P column k below the diagonal (row k+1 holds 1) and
// its scalar in S.tau[k]; H = Q T Q^+ with Q = H_0 H_1 ... H_{n-2},
// H_k = I - tau_k v_k v_k^+.
template <int NP>
__device__ void wave_tridiag(WaveLds<NP>& S, int n, double& d_lane, double& e_lane) {
    constexpr int LD = WaveLds<NP>::LD;
    constexpr int HW = NP / 2;
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));  // recomputed here, not hoisted out of the k loop
    const int i = lane >> 1, h = lane & 1;
    const bool row_ok = i < n;
    // reciprocal: hardware estimate and one Newton step
    auto rcp = [](double x) {
        const double r = __builtin_amdgcn_rcp(x);
        return fma(r, fma(-x, r, 1.0), r);
    };
    double2 a[HW];
#pragma unroll
    for (int jj = 0; jj < HW; ++jj)
        a[jj] = (row_ok && 2 * jj + h < n) ? S.P[i * LD + 2 * jj + h] : c_make(0.0, 0.0);
    d_lane = 0.0;
    e_lane = 0.0;
    for (int k = 0; k < n - 1; ++k) {
        const int hk = k & 1, jk = k >> 1;  // lane half and slot holding column k
        // a[jk]: a wave-uniform branch picks the group of four slots, a select the slot
        double2 xk = c_make(0.0, 0.0);
#pragma unroll
        for (int gq = 0; gq < HW / 4; ++gq) {
            if ((jk >> 2) == gq) {
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if ((jk & 3) == t) xk = a[4 * gq + t];
            }
        }
        const bool own = (h == hk);
        const double2 xp = c_make(dpp_xor1(xk.x), dpp_xor1(xk.y));
        const double2 x = own ? xk : xp;  // A[i][k] in both lanes of row i
        const int src = 2 * (k + 1) + hk;
        const double2 alpha = c_make(lane_read(xk.x, src), lane_read(xk.y, src));
        const double dk = lane_read(xk.x, 2 * k + hk);
        const double xn2 = wave_sum((own && i > k + 1 && i < n) ? (x.x * x.x + x.y * x.y) : 0.0);
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
            // 1 / (alpha - beta)
            const double ar = alpha.x - beta, ai = alpha.y;
            const double den = rcp(ar * ar + ai * ai);
            scal = c_make(ar * den, -ai * den);
        }
        double2 v = c_make(0.0, 0.0);
        if (i == k + 1)
            v = c_make(1.0, 0.0);
        else if (i > k + 1 && i < n)
            v = c_mul(x, scal);
        if (lane == k) {
            d_lane = dk;
            e_lane = beta;
        }
        // the reflector replaces column k below the diagonal
#pragma unroll
        for (int gq = 0; gq < HW / 4; ++gq) {
            if ((jk >> 2) == gq) {
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (own && (jk & 3) == t && i > k) a[4 * gq + t] = v;
            }
        }
        if (lane == 0) S.tau[k] = tau;
        if (h == 0 && i < NP) S.vv[i] = v;
        __syncthreads();
        if (tau.x == 0.0 && tau.y == 0.0) continue;
        // p = A v (row i), the two halves combined within the lane pair; v is read
        // whole (broadcast reads, one wait) and only the live groups are multiplied
        double2 vc[HW];
#pragma unroll
        for (int jj = 0; jj < HW; ++jj) vc[jj] = S.vv[2 * jj + h];
        double2 p = c_make(0.0, 0.0);
#pragma unroll
        for (int gq = 0; gq < HW / 4; ++gq) {
            if (8 * gq + 7 > k) {  // some column of this group of four slots is still live
#pragma unroll
                for (int t = 0; t < 4; ++t) p = c_fma(a[4 * gq + t], vc[4 * gq + t], p);
            }
        }
        p = c_make(p.x + dpp_xor1(p.x), p.y + dpp_xor1(p.y));
        const double mu = wave_sum(h == 0 ? (v.x * p.x + v.y * p.y) : 0.0);  // v^+ p (real)
        const double t2 = 0.5 * (tau.x * tau.x + tau.y * tau.y) * mu;
        double2 w = c_sub(c_mul(tau, p), c_scale(t2, v));
        if (!(i > k && i < n)) w = c_make(0.0, 0.0);
        if (h == 0 && i < NP) S.wv[i] = w;
        __syncthreads();
        // A <- A - v w^+ - w v^+ (v_c = w_c = 0 for c <= k keeps the stored reflectors)
        double2 wc[HW];
#pragma unroll
        for (int jj = 0; jj < HW; ++jj) wc[jj] = S.wv[2 * jj + h];
#pragma unroll
        for (int gq = 0; gq < HW / 4; ++gq) {
            if (8 * gq + 7 > k) {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int jj = 4 * gq + t;
                    a[jj] = c_rank2c(a[jj], v, wc[jj], w, vc[jj]);
                }
            }
        }
        __syncthreads();
    }
    {
        const int hl = (n - 1) & 1, jl = (n - 1) >> 1;
        double2 last = c_make(0.0, 0.0);
#pragma unroll
        for (int jj = 0; jj < HW; ++jj)
            if (jj == jl) last = a[jj];
        const double dl = lane_read(last.x, 2 * (n - 1) + hl);
        if (lane == n - 1) {
            d_lane = dl;
            e_lane = 0.0;
        }
    }
    // reflectors back to LDS for the back-transformation, with zeros on and above
    // the diagonal and in the padding rows, so that column k of S.P is v_k
    // exactly (no masking of its rows when it is applied)
    if (i < NP) {
#pragma unroll
        for (int jj = 0; jj < HW; ++jj)
            S.P[i * LD + 2 * jj + h] = (row_ok && 2 * jj + h < i) ? a[jj] : c_make(0.0, 0.0);
    }
    __syncthreads();
}

// Implicit QL with shifts on (d, e), one element per lane; accumulates the
// rotations into Z (real parts of S.U, identity on entry, lane = row).
// Returns false if some eigenvalue needed more than max_iter iterations.
template <int NP>
__device__ bool wave_ql(WaveLds<NP>& S, int n, double& d_lane, double& e_lane, int max_iter) {
    constexpr int LD = WaveLds<NP>::LD;
    const int lane = threadIdx.x & 63;
    bool ok = true;
    double f = 0.0, tst1 = 0.0;
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        {
            const double dl = lane_read(d_lane, l), el = lane_read(e_lane, l);
            tst1 = fmax(tst1, fabs(dl) + fabs(el));
        }
        for (;;) {
            const bool small = (lane >= l) && (lane < n) && (tst1 + fabs(e_lane) == tst1);
            const unsigned long long mask = __ballot(small);
            if (mask == 0ull) {  // only possible with NaN input: e_{n-1} = 0 always qualifies
                ok = false;
                break;
            }
            const int m = __ffsll((long long)mask) - 1;
            if (m <= l) break;
            if (++iter > max_iter) {
                ok = false;
                break;
            }
            // shift from the leading 2x2 block
            const double g0 = lane_read(d_lane, l);
            const double el = lane_read(e_lane, l);
            const double dnext = lane_read(d_lane, l + 1);
            double p = (dnext - g0) / (2.0 * el);
            double r = sqrt(p * p + 1.0);
            const double pr = p + copysign(r, p);
            const double new_dl = el / pr;
            const double dl1 = el * pr;
            double h = g0 - new_dl;
            if (lane >= l + 2 && lane < n) d_lane -= h;
            if (lane == l) d_lane = new_dl;
            if (lane == l + 1) d_lane = dl1;
            f += h;
            // QL sweep, i = m-1 down to l
            p = lane_read(d_lane, m);
            double c = 1.0, c2 = 1.0, c3 = 1.0, s = 0.0, s2 = 0.0;
            const double el1 = lane_read(e_lane, l + 1);
            for (int i = m - 1; i >= l; --i) {
                c3 = c2;
                c2 = c;
                s2 = s;
                const double ei = lane_read(e_lane, i);
                const double di = lane_read(d_lane, i);
                const double g = c * ei;
                h = c * p;
                r = sqrt(p * p + ei * ei);
                const double e_ip1 = s * r;
                const double inv = 1.0 / r;
                s = ei * inv;
                c = p * inv;
                p = c * di - s * g;
                const double d_ip1 = h + s * (c * g + s * di);
                if (lane == i + 1) {
                    e_lane = e_ip1;
                    d_lane = d_ip1;
                }
                if (lane == 0) {
                    S.cs[2 * i] = c;
                    S.cs[2 * i + 1] = s;
                }
            }
            p = -s * s2 * c3 * el1 * el / dl1;
            if (lane == l) {
                e_lane = s * p;
                d_lane = c * p;
            }
            __syncthreads();
            // apply the sweep to Z: rotation i mixes columns i and i+1
            if (lane < n) {
                double carry = S.U[lane * LD + m].x;
                for (int i = m - 1; i >= l; --i) {
                    const double ci = S.cs[2 * i], si = S.cs[2 * i + 1];
                    const double zi = S.U[lane * LD + i].x;
                    S.U[lane * LD + i + 1].x = si * zi + ci * carry;
                    carry = ci * zi - si * carry;
                }
                S.U[lane * LD + l].x = carry;
            }
            __syncthreads();
        }
        if (lane == l) d_lane += f;
        if (!ok) break;
    }
    return ok;
}

// Eigenvalues of the real symmetric tridiagonal matrix (d, e) in S.de2, lanes
// 2j and 2j+1 both returning eigenvalue j (ascending).  Each pass evaluates the
// Sturm sequence q_i = (d_i - x) - e_{i-1}^2 / q_{i-1} at one point per lane:
// the number of negative q_i is the number of eigenvalues below x, and, when
// asked for, the same recurrence gives S = d/dx log|det(T - x I)| = sum q_i'/q_i
// with q_i' = -1 + e_{i-1}^2 q_{i-1}' / q_{i-1}^2, so x - 1/S is the Newton step
// on det(T - x I).  Every lane pair keeps a bracket lo <= lambda_j < hi with
// the counts at its ends and, per pass:
//  * while lambda_j is not the only eigenvalue in the bracket: trisection (the
//    two lanes take the points at one and two thirds);
//  * once it is: lane 0 takes the Newton point of the previous pass, lane 1 the
//    bracket's midpoint (so the bracket at least halves every pass);
//  * a Newton step below the tolerance 4 eps max|lambda| is accepted only after
//    a verifying pass finds lambda_j between c - 2 tol and c + 2 tol by counts.
// The counts decide everything, as in plain bisection, so a poor derivative
// (cancellation near an eigenvalue of a leading submatrix) can cost passes but
// not accuracy.  Well-separated spectra finish in about a third of the passes of
// trisection to the same tolerance; clustered ones fall back to trisection.
template <int NP>
__device__ double wave_bisect(const WaveLds<NP>& S, int n, double glo, double ghi, double pivmin) {
    constexpr int kMaxPasses = 96;
    const int lane = threadIdx.x & 63;
    const int j = lane >> 1;
    const int half = lane & 1;
    auto rcp = [](double q) {
        const double r = __builtin_amdgcn_rcp(q);
        return fma(r, fma(-q, r, 1.0), r);
    };
    // the matrix in registers; rows past n decouple (e = 0) and never count (d huge)
    double dv[NP], e2v[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const double2 de = S.de2[i];
        dv[i] = (i < n) ? de.x : 1e300;
        e2v[i] = (i < n) ? de.y * de.y : 0.0;
    }
    const double scale = fmax(fabs(glo), fabs(ghi));
    const double tol = 4.0 * 2.220446049250313e-16 * scale + 1e-300;
    double lo = glo, hi = ghi, cand = 0.0, lam = ghi;
    int clo = 0, chi = n;
    bool done = j >= n, has = false, ver = false;
    for (int pass = 0; pass < kMaxPasses; ++pass) {
        if (__ballot(!done) == 0ull) break;
        const bool iso = (clo == j) && (chi == j + 1);
        const double w = hi - lo;
        double x;
        if (ver)
            x = half ? cand + 2.0 * tol : cand - 2.0 * tol;
        else if (iso && has)
            x = half ? lo + 0.5 * w : cand;
        else
            x = lo + (double)(half + 1) * (w * (1.0 / 3.0));
        const bool need_d = __ballot(!done && iso && !ver) != 0ull;  // wave-uniform
        int cnt = 0;
        double sd = 0.0;
        if (need_d) {
            double q = 1.0, qd = 0.0;
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const double e2p = (i > 0) ? e2v[i - 1] : 0.0;
                const double rq = rcp(q);
                sd = fma(qd, rq, sd);  // q'_{i-1} / q_{i-1}
                const double t = e2p * rq;
                double qi = (dv[i] - x) - t;
                if (fabs(qi) < pivmin) qi = -pivmin;
                qd = fma(t * rq, qd, -1.0);
                cnt += (qi < 0.0) ? 1 : 0;
                q = qi;
            }
            sd = fma(qd, rcp(q), sd);
        } else {
            double q = 1.0;
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const double e2p = (i > 0) ? e2v[i - 1] : 0.0;
                double qi = fma(-e2p, rcp(q), dv[i] - x);
                if (fabs(qi) < pivmin) qi = -pivmin;
                cnt += (qi < 0.0) ? 1 : 0;
                q = qi;
            }
        }
        // both lanes of the pair see both points in the same order
        const double xo = dpp_xor1(x), so = dpp_xor1(sd);
        const int co = __builtin_amdgcn_update_dpp(0, cnt, 0xB1, 0xF, 0xF, false);
        const double x0 = half ? xo : x, x1 = half ? x : xo;
        const double s0 = half ? so : sd, s1 = half ? sd : so;
        const int c0 = half ? co : cnt, c1 = half ? cnt : co;
        if (done) continue;
        if (ver && c0 <= j && c1 > j) {  // lambda_j within 2 tol of the Newton value
            done = true;
            lam = cand;
            continue;
        }
        if (c0 <= j && x0 > lo) { lo = x0; clo = c0; }
        if (c1 <= j && x1 > lo) { lo = x1; clo = c1; }
        if (c0 > j && x0 < hi) { hi = x0; chi = c0; }
        if (c1 > j && x1 < hi) { hi = x1; chi = c1; }
        const bool was_ver = ver;
        ver = false;
        has = false;
        if (need_d && !was_ver) {
            // Newton points from both evaluations; keep the shorter step in the bracket
            const double na = x0 - 1.0 / s0, nb = x1 - 1.0 / s1;
            const bool ina = (na >= lo - tol) && (na <= hi + tol);
            const bool inb = (nb >= lo - tol) && (nb <= hi + tol);
            const double sta = fabs(na - x0), stb = fabs(nb - x1);
            const bool pb = inb && (!ina || stb < sta);
            if (ina || inb) {
                const double c = pb ? nb : na;
                const double st = pb ? stb : sta;
                cand = fmin(fmax(c, lo), hi);
                if ((clo == j) && (chi == j + 1) && st <= tol)
                    ver = true;
                else
                    has = (c > lo) && (c < hi);
            }
        }
        if (!ver && hi - lo <= tol) {
            done = true;
            lam = 0.5 * (lo + hi);
        }
    }
    if (!done) lam = 0.5 * (lo + hi);
    return lam;
}

// Eigenvector of the tridiagonal matrix for an isolated eigenvalue lam by the
// twisted factorisation of T - lam I: forward pivots dp, backward pivots dm,
// twist index r = argmin |dp_r + dm_r - (d_r - lam)|, then z_r = 1 and the two
// one-sided recurrences.  The lane keeps the rows of parity h of the
// normalised vector: u[jj] = z[2 jj + h].
template <int NP>
__device__ void wave_twisted(const WaveLds<NP>& S, int n, double& lam, double pivmin, int h,
                             double2 (&u)[NP / 2]) {
    // 1/q: hardware estimate plus one Newton step (|q| >= pivmin keeps it finite)
    auto rcp = [](double q) {
        const double r = __builtin_amdgcn_rcp(q);
        return fma(r, fma(-q, r, 1.0), r);
    };
    double dp[NP], dm[NP];
    {
        double q = 1.0, e2prev = 0.0;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const double2 de = S.de2[i];
            double qi = (de.x - lam) - e2prev * rcp(q);
            if (fabs(qi) < pivmin) qi = -pivmin;
            dp[i] = qi;
            q = qi;
            e2prev = de.y * de.y;
        }
    }
    {
        double q = 1.0;
#pragma unroll
        for (int i = NP - 1; i >= 0; --i) {
            const double2 de = S.de2[i];
            double qi = (de.x - lam) - ((i < n - 1) ? de.y * de.y * rcp(q) : 0.0);
            if (fabs(qi) < pivmin) qi = -pivmin;
            dm[i] = qi;
            q = qi;
        }
    }
    int r = 0;
    double best = 1e308, gam = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        if (i < n) {
            const double g = dp[i] + dm[i] - (S.de2[i].x - lam);
            if (fabs(g) < best) {
                best = fabs(g);
                gam = g;
                r = i;
            }
        }
    }
    // z_r = 1; below the twist z_i = -(e_i / dp_i) z_{i+1} (kept in dp_i),
    // above it z_i = -(e_{i-1} / dm_i) z_{i-1} (kept in dm_i)
#pragma unroll
    for (int i = NP - 2; i >= 0; --i) {
        const double zn = (i + 1 == r) ? 1.0 : dp[i + 1];
        const double v = -(S.de2[i].y * rcp(dp[i])) * zn;
        if (i < r) dp[i] = v;
    }
#pragma unroll
    for (int i = 1; i < NP; ++i) {
        const double zp = (i - 1 == r) ? 1.0 : dm[i - 1];
        const double v = -(S.de2[i - 1].y * rcp(dm[i])) * zp;
        if (i > r) dm[i] = (i < n) ? v : 0.0;
    }
    double nrm = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const double zi = (i < r) ? dp[i] : ((i == r) ? 1.0 : dm[i]);
        nrm += zi * zi;
    }
    // (T - lam) z = gam e_r with z_r = 1: the Rayleigh quotient is lam + gam / |z|^2
    lam += gam / nrm;
    const double inv = 1.0 / sqrt(nrm);
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const double zi = (i < r) ? dp[i] : ((i == r) ? 1.0 : dm[i]);
        if ((i & 1) == h) u[i >> 1] = c_make(zi * inv, 0.0);
    }
}

// U <- H_0 H_1 ... H_{n-2} Z in registers: lane 2c + h holds rows 2 jj + h
// of column c in u[jj] (Z on entry); the reflectors are read from S.P
// (column k, zero on and above the diagonal and in the padding rows) as
// broadcasts, and groups of four slots whose eight rows are all above the
// reflector are skipped.
template <int NP>
__device__ void wave_backtransform(const WaveLds<NP>& S, int n, double2 (&u)[NP / 2]) {
    constexpr int LD = WaveLds<NP>::LD;
    constexpr int HW = NP / 2;
    const int h = threadIdx.x & 1;
    for (int k = n - 2; k >= 0; --k) {
        const double2 tau = S.tau[k];
        if (tau.x == 0.0 && tau.y == 0.0) continue;
        double2 vr[HW];
        double2 y = c_make(0.0, 0.0);  // v^+ u over this lane's rows of the column
#pragma unroll
        for (int gq = 0; gq < HW / 4; ++gq) {
#pragma unroll
            for (int t = 0; t < 4; ++t) vr[4 * gq + t] = c_make(0.0, 0.0);
            if (8 * gq + 7 > k) {  // some row of this group of four slots is below the reflector's top
#pragma unroll
                for (int t = 0; t < 4; ++t) vr[4 * gq + t] = S.P[(2 * (4 * gq + t) + h) * LD + k];
#pragma unroll
                for (int t = 0; t < 4; ++t) y = c_fmac(vr[4 * gq + t], u[4 * gq + t], y);
            }
        }
        y = c_make(y.x + dpp_xor1(y.x), y.y + dpp_xor1(y.y));
        const double2 ty = c_mul(tau, y);
#pragma unroll
        for (int gq = 0; gq < HW / 4; ++gq)
            if (8 * gq + 7 > k) {
#pragma unroll
                for (int t = 0; t < 4; ++t) u[4 * gq + t] = c_fnma(vr[4 * gq + t], ty, u[4 * gq + t]);
            }
    }
}

// Upper triangle (diagonal included) of an NP x NP matrix packed row by row:
// row i starts at s(i) = i NP - i (i - 1) / 2.  Element e -> (i, j), i <= j.
template <int NP>
__device__ __forceinline__ void upper_index(int e, int& i, int& j) {
    constexpr float b = 2.0f * NP + 1.0f;
    int r = (int)(0.5f * (b - sqrtf(b * b - 8.0f * (float)e)));
    auto start = [](int q) { return q * NP - (q * (q - 1)) / 2; };
    if (start(r) > e) --r;
    else if (start(r + 1) <= e) ++r;
    i = r;
    j = r + (e - start(r));
}

// M = U^+ v U for one velocity; lane (i = lane/2, half h) returns row i,
// columns [h NP/2, (h+1) NP/2) of M in M[].  v_il = sum_rho coef_rho T[rho][i][l],
// coef = e^{i k0 rho} (times i rho for v_x).  W = v U passes through S.P.
template <int NP>
__device__ void wave_velocity(WaveLds<NP>& S, int n, int nR0, const double2* __restrict__ T,
                              const int* __restrict__ r0, bool is_x, double2 (&M)[NP / 2],
                              const double* sw = nullptr) {
    constexpr int LD = WaveLds<NP>::LD;
    constexpr int HW = NP / 2;
    const int lane = threadIdx.x & 63;
    const int i = lane >> 1;
    const int j0 = (lane & 1) * HW;
    const long long nn = (long long)n * n;
    double2 acc[HW];
#pragma unroll
    for (int jj = 0; jj < HW; ++jj) acc[jj] = c_make(0.0, 0.0);
    if (i < n) {
        for (int l = 0; l < n; ++l) {
            double2 v = c_make(0.0, 0.0);
            for (int rho = 0; rho < nR0; ++rho) {
                double2 cf = S.ph[rho];
                if (is_x) cf = c_scale((double)r0[rho], c_i(cf));
                v = c_fma(cf, T[(long long)rho * nn + i * n + l], v);
            }
            if (sw) v = c_scale(0.5 * (sw[i] + sw[l]), v);  // spin current (s v + v s)/2
#pragma unroll
            for (int jj = 0; jj < HW; ++jj) acc[jj] = c_fma(v, S.U[l * LD + j0 + jj], acc[jj]);
        }
    }
    __syncthreads();
    if (i < n) {
#pragma unroll
        for (int jj = 0; jj < HW; ++jj)
            if (j0 + jj < n) S.P[i * LD + j0 + jj] = acc[jj];
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < HW; ++jj) acc[jj] = c_make(0.0, 0.0);
    if (i < n) {
        for (int l = 0; l < n; ++l) {
            const double2 u = S.U[l * LD + i];
#pragma unroll
            for (int jj = 0; jj < HW; ++jj)
                if (j0 + jj < n) acc[jj] = c_fmac(u, S.P[l * LD + j0 + jj], acc[jj]);
        }
    }
#pragma unroll
    for (int jj = 0; jj < HW; ++jj) M[jj] = acc[jj];
    __syncthreads();
}

// v (v_x if is_x, else v_y) into S.P, zero-padded to NP x NP:
// v_il = sum_rho coef_rho T[rho][i][l], coef = e^{i k0 rho} (times i rho for v_x).
// v is Hermitian (the hoppings are Hermitian-projected), so only the upper
// triangle is summed and the lower one is its mirror; consecutive lanes take
// consecutive elements of a row, so the loads stay coalesced.
template <int NP>
__device__ void wave_stage_velocity(WaveLds<NP>& S, int n, int nR0, const double2* __restrict__ T,
                                    const int* __restrict__ r0, bool is_x,
                                    const double* sw = nullptr) {
    constexpr int LD = WaveLds<NP>::LD;
    constexpr int NU = NP * (NP + 1) / 2;
    constexpr int PER = (NU + 63) / 64;
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));  // recomputed here, not hoisted out of the k loop
    const long long nn = (long long)n * n;
    double2 acc[PER];
    int off[PER];  // -1: padding
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = lane + 64 * q;
        int i, j;
        upper_index<NP>(e < NU ? e : 0, i, j);
        off[q] = (e < NU && j < n) ? i * n + j : -1;
        acc[q] = c_make(0.0, 0.0);
    }
    for (int rho = 0; rho < nR0; ++rho) {
        double2 cf = S.ph[rho];
        if (is_x) cf = c_scale((double)r0[rho], c_i(cf));
        const double2* Tr = T + (long long)rho * nn;
        // unconditional loads (padding from element 0, then zeroed): all in flight together
        double2 tv[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) tv[q] = Tr[off[q] >= 0 ? off[q] : 0];
#pragma unroll
        for (int q = 0; q < PER; ++q)
            acc[q] = c_fma(cf, (off[q] >= 0) ? tv[q] : c_make(0.0, 0.0), acc[q]);
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = lane + 64 * q;
        if (e < NU) {
            int i, j;
            upper_index<NP>(e, i, j);
            double2 v = acc[q];
            if (i == j) v.y = 0.0;
            // spin current (s v + v s)/2 for a diagonal s (zero past n: v is zero there)
            if (sw && j < n) v = c_scale(0.5 * (sw[i] + sw[j]), v);
            S.P[i * LD + j] = v;
            S.P[j * LD + i] = c_conj(v);
        }
    }
}

// The U operands of both products: u[kt][s][tc] = U[16 kt + g + 4 s][16 tc + c],
// g = lane / 16, c = lane % 16 (the B operand of k-step (kt, s) for column tile tc).
template <int NP>
__device__ void wave_load_uops(const WaveLds<NP>& S, double2 (&u)[NP / 16][4][NP / 16]) {
    constexpr int LD = WaveLds<NP>::LD, NT = NP / 16;
    const int lane = threadIdx.x & 63, g = lane >> 4, c16 = lane & 15;
#pragma unroll
    for (int kt = 0; kt < NT; ++kt)
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int tc = 0; tc < NT; ++tc) u[kt][s][tc] = S.U[(16 * kt + g + 4 * s) * LD + 16 * tc + c16];
}

// M = U^+ v U from the staged v (S.P).  On return mr/mi[ti][tj][q] hold
// Re/Im M[16 ti + g + 4 q][16 tj + c].
//   X = v U:   k-step (kt, s) takes contraction index 16 kt + g + 4 s from lane group g;
//   M = X^+ U: with the same contraction order, the A operand of lane l at
//              k-step (kt, s) for row tile ti is conj(X[16 kt + g + 4 s][16 ti + c]),
//              which is element s of the lane's own X tile (kt, ti).
template <int NP>
__device__ void wave_rotate_mfma(const WaveLds<NP>& S, const double2 (&u)[NP / 16][4][NP / 16],
                                 v4d (&mr)[NP / 16][NP / 16], v4d (&mi)[NP / 16][NP / 16]) {
    constexpr int LD = WaveLds<NP>::LD, NT = NP / 16;
    const int lane = threadIdx.x & 63, g = lane >> 4, c16 = lane & 15;
    const v4d zero = {0.0, 0.0, 0.0, 0.0};
    v4d xr[NT][NT], xi[NT][NT];
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) {
            xr[a][b] = zero;
            xi[a][b] = zero;
            mr[a][b] = zero;
            mi[a][b] = zero;
        }
#pragma unroll
    for (int kt = 0; kt < NT; ++kt) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            double2 a[NT];
#pragma unroll
            for (int tr = 0; tr < NT; ++tr) a[tr] = S.P[(16 * tr + c16) * LD + 16 * kt + g + 4 * s];
            // (a_r + i a_i)(b_r + i b_i); independent accumulators back to back
#pragma unroll
            for (int tr = 0; tr < NT; ++tr)
#pragma unroll
                for (int tc = 0; tc < NT; ++tc) xr[tr][tc] = mfma16(a[tr].x, u[kt][s][tc].x, xr[tr][tc]);
#pragma unroll
            for (int tr = 0; tr < NT; ++tr)
#pragma unroll
                for (int tc = 0; tc < NT; ++tc) xi[tr][tc] = mfma16(a[tr].x, u[kt][s][tc].y, xi[tr][tc]);
#pragma unroll
            for (int tr = 0; tr < NT; ++tr)
#pragma unroll
                for (int tc = 0; tc < NT; ++tc) xr[tr][tc] = mfma16(-a[tr].y, u[kt][s][tc].y, xr[tr][tc]);
#pragma unroll
            for (int tr = 0; tr < NT; ++tr)
#pragma unroll
                for (int tc = 0; tc < NT; ++tc) xi[tr][tc] = mfma16(a[tr].y, u[kt][s][tc].x, xi[tr][tc]);
        }
    }
    // (x_r - i x_i)(b_r + i b_i)
#pragma unroll
    for (int kt = 0; kt < NT; ++kt) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int tj = 0; tj < NT; ++tj) mr[ti][tj] = mfma16(xr[kt][ti][s], u[kt][s][tj].x, mr[ti][tj]);
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int tj = 0; tj < NT; ++tj) mi[ti][tj] = mfma16(xr[kt][ti][s], u[kt][s][tj].y, mi[ti][tj]);
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int tj = 0; tj < NT; ++tj) mr[ti][tj] = mfma16(xi[kt][ti][s], u[kt][s][tj].y, mr[ti][tj]);
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int tj = 0; tj < NT; ++tj) mi[ti][tj] = mfma16(-xi[kt][ti][s], u[kt][s][tj].x, mi[ti][tj]);
        }
    }
}

// Omega_i = -2 sum_{j != i} Im(A_ij conj(B_ij)) g(E_i - E_j) into S.Om from the
// accumulator tiles of A and B (row i = 16 ti + g + 4 q, column j = 16 tj + c).
template <int NP>
__device__ void wave_curvature_mfma(WaveLds<NP>& S, int n, double eta2,
                                    const v4d (&ar)[NP / 16][NP / 16], const v4d (&ai)[NP / 16][NP / 16],
                                    const v4d (&br)[NP / 16][NP / 16], const v4d (&bi)[NP / 16][NP / 16],
                                    double* out) {
    constexpr int NT = NP / 16;
    const int lane = threadIdx.x & 63, g = lane >> 4, c16 = lane & 15;
    double om[NT][4];
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int q = 0; q < 4; ++q) om[ti][q] = 0.0;
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) {
        const int j = 16 * tj + c16;
        const double ej = (j < n) ? S.E[j] : 0.0;
#pragma unroll
        for (int ti = 0; ti < NT; ++ti)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 16 * ti + g + 4 * q;
                if (i < n && j < n && i != j) {
                    const double de = S.E[i] - ej;
                    const double den = de * de + eta2;
                    if (den > 0.0) {
                        const double qij = ai[ti][tj][q] * br[ti][tj][q] - ar[ti][tj][q] * bi[ti][tj][q];
                        om[ti][q] += qij / den;
                    }
                }
            }
    }
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double tot = row16_sum(om[ti][q]);
            const int i = 16 * ti + g + 4 * q;
            if (c16 == 0 && i < n) out[i] = -2.0 * tot;
        }
}

// The Hall tensor's extra LDS, placed right after WaveLds: the curvatures of the
// yz, zx and spin Hall pairs, and the spin diagonal of the k-point's model.
template <int NP>
struct WaveTensorLds {
    double Om2[3][NP];
    double spin[NP];
};

// An accumulator-layout matrix (element q of tile (ti, tj) is M[16 ti + g + 4 q][16 tj + c])
// written out in full to an LDS matrix with leading dimension LD.
template <int NP>
__device__ void wave_store_acc(double2* M, const v4d (&mr)[NP / 16][NP / 16],
                               const v4d (&mi)[NP / 16][NP / 16]) {
    constexpr int LD = WaveLds<NP>::LD, NT = NP / 16;
    const int lane = threadIdx.x & 63, g = lane >> 4, c16 = lane & 15;
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int tj = 0; tj < NT; ++tj)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                M[(16 * ti + g + 4 * q) * LD + 16 * tj + c16] = c_make(mr[ti][tj][q], mi[ti][tj][q]);
}

// out_i = -2 sum_{j != i} Im(P_ij conj(Q_ij)) g(E_i - E_j) with P in accumulator tiles
// and Q (Hermitian) read from the LDS matrix Qm at the same positions.
template <int NP>
__device__ void wave_curvature_lds(WaveLds<NP>& S, int n, double eta2,
                                   const v4d (&pr)[NP / 16][NP / 16], const v4d (&pi)[NP / 16][NP / 16],
                                   const double2* Qm, double* out) {
    constexpr int LD = WaveLds<NP>::LD, NT = NP / 16;
    const int lane = threadIdx.x & 63, g = lane >> 4, c16 = lane & 15;
    double om[NT][4];
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int q = 0; q < 4; ++q) om[ti][q] = 0.0;
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) {
        const int j = 16 * tj + c16;
        const double ej = (j < n) ? S.E[j] : 0.0;
#pragma unroll
        for (int ti = 0; ti < NT; ++ti)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 16 * ti + g + 4 * q;
                if (i < n && j < n && i != j) {
                    const double de = S.E[i] - ej;
                    const double den = de * de + eta2;
                    if (den > 0.0) {
                        const double2 qv = Qm[i * LD + j];
                        om[ti][q] += (pi[ti][tj][q] * qv.x - pr[ti][tj][q] * qv.y) / den;
                    }
                }
            }
    }
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double tot = row16_sum(om[ti][q]);
            const int i = 16 * ti + g + 4 * q;
            if (c16 == 0 && i < n) out[i] = -2.0 * tot;
        }
}

// Steps 1-2 at one k-point, one wavefront: H(k), its eigenvalues (S.E) and
// eigenvectors (S.U).  Returns false on QL non-convergence or non-finite values.
//
// v_x is built from the same loads of the pencil partial sums as H and parked
// in S.U until U takes its place, then moved to S.P; on return vx_in_p says
// whether S.P holds it (not after the QL path, which needs S.U for Z).
template <int NP>
__device__ bool wave_eigen(WaveLds<NP>& S, const ModelDev& md, const double2* __restrict__ T0,
                           const int* __restrict__ r0, int i0, int max_iter, bool& vx_in_p) {
    constexpr int LD = WaveLds<NP>::LD;
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));  // recomputed here, not hoisted out of the k loop
    const int n = md.n;
    const long long nn = (long long)n * n;
    if (lane < md.nR0) S.ph[lane] = unit_phase((long long)i0 * r0[lane], md.N0);
    __syncthreads();
    {
        // H and v_x from one pass over the upper triangles of the pencil partial
        // sums (both are Hermitian: the lower triangle is the mirror, so both are
        // exactly Hermitian), all loads of one rho in flight
        constexpr int NU = NP * (NP + 1) / 2;
        constexpr int PER = (NU + 63) / 64;
        double2 acc[PER], accx[PER];
        int off[PER];  // -1: padding
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = lane + 64 * q;
            int i, j;
            upper_index<NP>(e < NU ? e : 0, i, j);
            off[q] = (e < NU && j < n) ? i * n + j : -1;
            acc[q] = c_make(0.0, 0.0);
            accx[q] = c_make(0.0, 0.0);
        }
        for (int rho = 0; rho < md.nR0; ++rho) {
            const double2 ph = S.ph[rho];
            const double2 cf = c_scale((double)r0[rho], c_i(ph));
            const double2* Tr = T0 + (long long)rho * nn;
            // every lane loads (padding from element 0, then zeroed), so that the
            // loads are not each behind a branch and a wait of their own
            double2 tv[PER];
#pragma unroll
            for (int q = 0; q < PER; ++q) tv[q] = Tr[off[q] >= 0 ? off[q] : 0];
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const double2 t = (off[q] >= 0) ? tv[q] : c_make(0.0, 0.0);
                acc[q] = c_fma(t, ph, acc[q]);
                accx[q] = c_fma(cf, t, accx[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = lane + 64 * q;
            if (e < NU) {
                int i, j;
                upper_index<NP>(e, i, j);
                double2 h = acc[q], x = accx[q];
                if (i == j) {
                    h.y = 0.0;
                    x.y = 0.0;
                }
                if (off[q] >= 0) {
                    S.P[i * LD + j] = h;
                    S.P[j * LD + i] = c_conj(h);
                }
                S.U[i * LD + j] = x;
                S.U[j * LD + i] = c_conj(x);
            }
        }
    }
    vx_in_p = true;
    __syncthreads();
    double d_lane, e_lane;
    wave_tridiag<NP>(S, n, d_lane, e_lane);
    if (lane < NP) S.de2[lane] = (lane < n) ? c_make(d_lane, e_lane) : c_make(0.0, 0.0);
    __syncthreads();
    // Gershgorin interval and the pivot floor of the Sturm sequences
    const double e_prev = (lane > 0 && lane < n) ? S.de2[lane - 1].y : 0.0;
    const double rad = (lane < n) ? fabs(e_prev) + fabs(e_lane) : 0.0;
    const double glo = wave_min(lane < n ? d_lane - rad : 1e300);
    const double ghi = wave_max(lane < n ? d_lane + rad : -1e300);
    const double emax = wave_max(lane < n ? fabs(e_lane) : 0.0);
    const double pivmin = 1e-290 * fmax(1.0, emax * emax);
    bool ok = true;
    const double lam2 = wave_bisect<NP>(S, n, glo, ghi, pivmin);  // lanes 2j, 2j+1: eigenvalue j
    constexpr int HW = NP / 2;
    const int c = lane >> 1, h = lane & 1;
    const double lnext = __shfl_down(lam2, 2, 64);
    const double span = fmax(fabs(glo), fabs(ghi));
    const bool close = (c < n - 1) && (lnext - lam2 < 1e-3 * span);
    double2 u[HW];
    // (the debug iteration cap sends every k-point through the iterative path)
    if (__ballot(close) == 0ull && max_iter > 1) {
        // isolated eigenvalues: one twisted factorisation per lane pair
#pragma unroll
        for (int jj = 0; jj < HW; ++jj) u[jj] = c_make(0.0, 0.0);
        if (c < n) {
            double lam_c = lam2;
            wave_twisted<NP>(S, n, lam_c, pivmin, h, u);
            if (h == 0) S.E[c] = lam_c;
            if (!isfinite(lam_c)) ok = false;
        }
    } else {
        // a cluster: implicit QL with accumulated rotations (Z in S.U, lane = row)
        vx_in_p = false;
        for (int e = lane; e < n * n; e += 64) {
            const int i = e / n, j = e - (e / n) * n;
            S.U[i * LD + j] = c_make(i == j ? 1.0 : 0.0, 0.0);
        }
        __syncthreads();
        ok = wave_ql<NP>(S, n, d_lane, e_lane, max_iter);
        if (lane < n) S.E[lane] = d_lane;
        if (__ballot(lane < n && !isfinite(d_lane)) != 0ull) ok = false;
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < HW; ++jj) {
            const int r = 2 * jj + h;
            u[jj] = (c < n && r < n) ? c_make(S.U[r * LD + c].x, 0.0) : c_make(0.0, 0.0);
        }
    }
    if (__ballot(!ok) != 0ull) ok = false;
    wave_backtransform<NP>(S, n, u);
    __syncthreads();
    if (vx_in_p) {
        // the reflectors are spent: v_x moves from S.U to S.P
        constexpr int PER = NP * NP / 64;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = lane + 64 * q;
            const int idx = (e / NP) * LD + (e % NP);
            S.P[idx] = S.U[idx];
        }
        __syncthreads();
    }
    if (c < NP) {
#pragma unroll
        for (int jj = 0; jj < HW; ++jj) {
            const int r = 2 * jj + h;
            S.U[r * LD + c] = (c < n && r < n) ? u[jj] : c_make(0.0, 0.0);
        }
    }
    __syncthreads();
    return ok;
}

// ---------------------------------------------------------------------------
// k_forward_wave: steps 1-4 with one wavefront per workgroup (n <= NP <= 32).
// TENSOR: also v_z and the spin current (s v_x + v_x s)/2 rotated into the
// eigenbasis, four curvatures per band (pairs (v_x, v_y), (v_y, v_z), (v_z, v_x),
// (Js_x, v_y)) and four Fermi sums per level.
// ---------------------------------------------------------------------------
template <int NP, bool TENSOR>
__global__ __launch_bounds__(64) void k_forward_wave(FwdLaunch a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    WaveLds<NP>& S = *reinterpret_cast<WaveLds<NP>*>(smem_raw);
    WaveTensorLds<NP>& ST = *reinterpret_cast<WaveTensorLds<NP>*>(smem_raw + sizeof(WaveLds<NP>));
    constexpr int LD = WaveLds<NP>::LD;
    constexpr int HW = NP / 2;
    constexpr int NT = NP / 16;
    constexpr int NC = TENSOR ? 4 : 1;
    const int lane = threadIdx.x & 63;
    const double eta2 = a.eta * a.eta;
    const int max_iter = a.max_sweeps >= kMaxSweeps ? 30 : 1;
    const double2* tbuf = reinterpret_cast<const double2*>(a.tbuf);
    const bool with_spin = TENSOR && a.spin != nullptr;
    // U's padding (rows and columns n..NP-1) is never written below: keep it finite
    for (int e = lane; e < NP * LD; e += 64) S.U[e] = c_make(0.0, 0.0);
    __syncthreads();
    int probe = 0;
    for (;;) {
        int item = 0;
        if (lane == 0) item = queue_take(a.queue, a.item_count, probe);
        item = __builtin_amdgcn_readfirstlane(item);
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
        double* part = a.partial + (long long)it.slot * a.nF * NC;
        if constexpr (TENSOR) {
            if (lane < NP) ST.spin[lane] = (with_spin && lane < n) ? a.spin[md.orb_off + lane] : 0.0;
            if (lane < NP) {
                ST.Om2[0][lane] = 0.0;
                ST.Om2[1][lane] = 0.0;
                ST.Om2[2][lane] = 0.0;
            }
        }
        for (int kk = 0; kk < it.count; ++kk) {
            bool vx_in_p;
            const bool ok = wave_eigen<NP>(S, md, T0, r0, it.i0 + kk, max_iter, vx_in_p);
            if (!ok && lane == 0) atomicOr(a.status, kStatNoConv);
            if constexpr (NT >= 1) {
                // A = U^+ v_x U, B = U^+ v_y U on the matrix cores
                double2 u[NT][4][NT];
                wave_load_uops<NP>(S, u);
                if (!vx_in_p) {
                    wave_stage_velocity<NP>(S, n, md.nR0, T0, r0, true);
                    __syncthreads();
                }
                v4d ar[NT][NT], ai[NT][NT], br[NT][NT], bi[NT][NT];
                wave_rotate_mfma<NP>(S, u, ar, ai);
                __syncthreads();
                wave_stage_velocity<NP>(S, n, md.nR0, T1, r0, false);
                __syncthreads();
                wave_rotate_mfma<NP>(S, u, br, bi);
                wave_curvature_mfma<NP>(S, n, eta2, ar, ai, br, bi, S.Om);
                if constexpr (TENSOR) {
                    // U sits in registers now: S.U keeps A for the (v_z, v_x) pair
                    wave_store_acc<NP>(S.U, ar, ai);
                    if (with_spin) {
                        __syncthreads();
                        wave_stage_velocity<NP>(S, n, md.nR0, T0, r0, true, ST.spin);
                        __syncthreads();
                        wave_rotate_mfma<NP>(S, u, ar, ai);  // D = U^+ Js_x U
                        wave_curvature_mfma<NP>(S, n, eta2, ar, ai, br, bi, ST.Om2[2]);
                    }
                    __syncthreads();
                    wave_stage_velocity<NP>(S, n, md.nR0, T2, r0, false);
                    __syncthreads();
                    wave_rotate_mfma<NP>(S, u, ar, ai);  // C = U^+ v_z U
                    wave_curvature_mfma<NP>(S, n, eta2, br, bi, ar, ai, ST.Om2[0]);
                    wave_curvature_lds<NP>(S, n, eta2, ar, ai, S.U, ST.Om2[1]);
                }
            } else {
                double2 Ma[HW], Mb[HW];
                wave_velocity<NP>(S, n, md.nR0, T0, r0, true, Ma);
                wave_velocity<NP>(S, n, md.nR0, T1, r0, false, Mb);
                // Omega_i = -2 sum_{j != i} Im(P_ij Q_ji) g(E_i - E_j), Q_ji = conj(Q_ij)
                const int i = lane >> 1;
                const int j0 = (lane & 1) * HW;
                auto curv = [&](const double2 (&P)[HW], const double2 (&Q)[HW], double* out) {
                    double om = 0.0;
                    if (i < n) {
                        const double ei = S.E[i];
#pragma unroll
                        for (int jj = 0; jj < HW; ++jj) {
                            const int j = j0 + jj;
                            if (j < n && j != i) {
                                const double de = ei - S.E[j];
                                const double den = de * de + eta2;
                                if (den > 0.0) {
                                    const double q = P[jj].y * Q[jj].x - P[jj].x * Q[jj].y;
                                    om += q / den;
                                }
                            }
                        }
                    }
                    om += __shfl_xor(om, 1, 64);
                    if (i < n && (lane & 1) == 0) out[i] = -2.0 * om;
                };
                curv(Ma, Mb, S.Om);
                if constexpr (TENSOR) {
                    double2 Mc[HW];
                    wave_velocity<NP>(S, n, md.nR0, T2, r0, false, Mc);
                    curv(Mb, Mc, ST.Om2[0]);
                    curv(Mc, Ma, ST.Om2[1]);
                    if (with_spin) {
                        wave_velocity<NP>(S, n, md.nR0, T0, r0, true, Mc, ST.spin);
                        curv(Mc, Mb, ST.Om2[2]);
                    }
                }
            }
            __syncthreads();
            const double ikT = (a.kT > 0.0) ? 1.0 / a.kT : 0.0;
            for (int j = lane; j < a.nF; j += 64) {
                const double efj = ef[j];
                double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
                for (int b = 0; b < n; ++b) {
                    const double f = occupation_ikt(S.E[b], efj, a.kT, ikT);
                    s0 += f * S.Om[b];
                    if constexpr (TENSOR) {
                        s1 += f * ST.Om2[0][b];
                        s2 += f * ST.Om2[1][b];
                        s3 += f * ST.Om2[2][b];
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
    (void)LD;
}

template <int NP, bool TENSOR>
static hipError_t launch_forward_wave_t(const FwdLaunch& L, hipStream_t s) {
    const size_t lds = sizeof(WaveLds<NP>) + (TENSOR ? sizeof(WaveTensorLds<NP>) : 0);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_forward_wave<NP, TENSOR>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    int grid = L.item_count < L.max_groups ? L.item_count : L.max_groups;
    hipLaunchKernelGGL((k_forward_wave<NP, TENSOR>), dim3(grid), dim3(64), lds, s, L);
    return hipGetLastError();
}

hipError_t launch_forward_wave(const FwdLaunch& L, hipStream_t s) {
    if (L.item_count <= 0) return hipSuccess;
    if (!L.queue) return hipErrorInvalidValue;
    switch (L.np) {
        case 8:
            return L.tensor ? launch_forward_wave_t<8, true>(L, s) : launch_forward_wave_t<8, false>(L, s);
        case 16:
            return L.tensor ? launch_forward_wave_t<16, true>(L, s) : launch_forward_wave_t<16, false>(L, s);
        case 32:
            return L.tensor ? launch_forward_wave_t<32, true>(L, s) : launch_forward_wave_t<32, false>(L, s);
        default:
            return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// k_adjoint_wave: reverse mode of steps 1-4 for one k-point per wavefront
// (n <= NP <= 32), every dense product on the matrix cores.  For
// L = sum_j sbar_j sigma_j and phi(E) = sum_j sbar_j f_j(E):
//   K_mq  = (phi_m - phi_q) g(E_m - E_q)          (real, antisymmetric)
//   Abar  = (i/N) K o B,  Bbar = -(i/N) K o A     (Hermitian)
//   D     = (K o B) A - (K o A) B,  X = (i/N)(D + D^+) = [Abar, A] + [Bbar, B]
//   Hbar' = X_mq / (E_m - E_q) off the diagonal; on the diagonal and for
//           pairs closer than delta, the divided-difference limit
//           (i/N) sum_p dK(x, E_p)/dx at x = (E_m + E_q)/2 (B_mp A_pq - A_mp B_pq)
//   Hbar  = U Hbar' U^+,  vbar_x = U Abar U^+,  vbar_y = U Bbar U^+
// stored per k-point (Hbar, vbar_x, vbar_y); a separate pass forms the
// block's pencil partials from them.  Every matrix is held in the
// accumulator layout: element q of lane l's tile (ti, tj) is
// M[16 ti + g + 4 q][16 tj + c].
// ---------------------------------------------------------------------------

// f(x) and f'(x) summed against sbar: one exponential per Fermi level
__device__ __forceinline__ void wave_phi_at(double x, const double* __restrict__ ef,
                                            const double* __restrict__ sb, int nF, double kT,
                                            double& phi, double& dphi) {
    double p = 0.0, d = 0.0;
    if (kT > 0.0) {
        const double ikT = 1.0 / kT;
#pragma unroll 4
        for (int j = 0; j < nF; ++j) {
            const double u = (x - ef[j]) * ikT;
            const double w = exp(-fabs(u));
            const double dd = 1.0 + w;
            double r = __builtin_amdgcn_rcp(dd);
            r = fma(r, fma(-dd, r, 1.0), r);
            const double f = (u > 0.0) ? w * r : r;
            p += sb[j] * f;
            d -= sb[j] * (w * r * r) * ikT;  // f (1 - f) / kT = w / (1 + w)^2 / kT
        }
    } else {
        for (int j = 0; j < nF; ++j) p += sb[j] * occupation(x, ef[j], kT);
    }
    phi = p;
    dphi = d;
}

// R = U M U^+ for Hermitian M (accumulator layout), with
// ua[kt][s][tr] = U[16 tr + c][16 kt + g + 4 s]:
//   Q = M U^+: A operand M[16 tr + c][kappa] = conj(M[kappa][16 tr + c]) (own element),
//              B operand conj(U[16 tc + c][kappa]) = conj(ua);
//   R = U Q:   A operand ua, B operand Q[kappa][16 tc + c] (own element).
template <int NP>
__device__ void wave_sandwich(const v4d (&mr)[NP / 16][NP / 16], const v4d (&mi)[NP / 16][NP / 16],
                              const double2 (&ua)[NP / 16][4][NP / 16], v4d (&rr)[NP / 16][NP / 16],
                              v4d (&ri)[NP / 16][NP / 16]) {
    constexpr int NT = NP / 16;
    const v4d zero = {0.0, 0.0, 0.0, 0.0};
    v4d qr[NT][NT], qi[NT][NT];
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) {
            qr[a][b] = zero;
            qi[a][b] = zero;
            rr[a][b] = zero;
            ri[a][b] = zero;
        }
    // Q = M U^+: (x_r - i x_i)(u_r - i u_i) with x = M[kappa][16 tr + c], u = U[16 tc + c][kappa]
#pragma unroll
    for (int kt = 0; kt < NT; ++kt) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int tr = 0; tr < NT; ++tr)
#pragma unroll
                for (int tc = 0; tc < NT; ++tc) qr[tr][tc] = mfma16(mr[kt][tr][s], ua[kt][s][tc].x, qr[tr][tc]);
#pragma unroll
            for (int tr = 0; tr < NT; ++tr)
#pragma unroll
                for (int tc = 0; tc < NT; ++tc) qi[tr][tc] = mfma16(-mr[kt][tr][s], ua[kt][s][tc].y, qi[tr][tc]);
#pragma unroll
            for (int tr = 0; tr < NT; ++tr)
#pragma unroll
                for (int tc = 0; tc < NT; ++tc) qr[tr][tc] = mfma16(-mi[kt][tr][s], ua[kt][s][tc].y, qr[tr][tc]);
#pragma unroll
            for (int tr = 0; tr < NT; ++tr)
#pragma unroll
                for (int tc = 0; tc < NT; ++tc) qi[tr][tc] = mfma16(-mi[kt][tr][s], ua[kt][s][tc].x, qi[tr][tc]);
        }
    }
    // R = U Q: (u_r + i u_i)(q_r + i q_i) with u = U[16 tr + c][kappa], q = Q[kappa][16 tc + c]
#pragma unroll
    for (int kt = 0; kt < NT; ++kt) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int tr = 0; tr < NT; ++tr)
#pragma unroll
                for (int tc = 0; tc < NT; ++tc) rr[tr][tc] = mfma16(ua[kt][s][tr].x, qr[kt][tc][s], rr[tr][tc]);
#pragma unroll
            for (int tr = 0; tr < NT; ++tr)
#pragma unroll
                for (int tc = 0; tc < NT; ++tc) ri[tr][tc] = mfma16(ua[kt][s][tr].x, qi[kt][tc][s], ri[tr][tc]);
#pragma unroll
            for (int tr = 0; tr < NT; ++tr)
#pragma unroll
                for (int tc = 0; tc < NT; ++tc) rr[tr][tc] = mfma16(-ua[kt][s][tr].y, qi[kt][tc][s], rr[tr][tc]);
#pragma unroll
            for (int tr = 0; tr < NT; ++tr)
#pragma unroll
                for (int tc = 0; tc < NT; ++tc) ri[tr][tc] = mfma16(ua[kt][s][tr].y, qr[kt][tc][s], ri[tr][tc]);
        }
    }
}

template <int NP>
__global__ __launch_bounds__(64) void k_adjoint_wave(WgLaunch a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    WaveLds<NP>& S = *reinterpret_cast<WaveLds<NP>*>(smem_raw);
    constexpr int LD = WaveLds<NP>::LD;
    constexpr int NT = NP / 16;
    static_assert(NT >= 1, "the matrix-core adjoint needs NP >= 16");
    const int lane = threadIdx.x & 63;
    const double eta2 = a.eta * a.eta;
    const double scl = (a.kT > 0.0) ? fmin(a.eta, a.kT) : a.eta;
    const double delta = 1e-5 * scl;
    const int max_iter = a.max_iter >= kMaxSweeps ? 30 : 1;
    const double2* tbuf = reinterpret_cast<const double2*>(a.tbuf);
    double2* xb = reinterpret_cast<double2*>(a.xbuf);
    const v4d zero = {0.0, 0.0, 0.0, 0.0};
    for (int e = lane; e < NP * LD; e += 64) S.U[e] = c_make(0.0, 0.0);
    __syncthreads();
    const int units = a.item_count * a.unit_parts;
    int probe = 0;
    for (;;) {
        int unit = 0;
        if (lane == 0) unit = queue_take(a.queue, units, probe);
        unit = __builtin_amdgcn_readfirstlane(unit);
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
            // lane-derived values recomputed per k-point rather than hoisted out of the loop
            int lane_k = threadIdx.x & 63;
            asm volatile("" : "+v"(lane_k));
            const int lane = lane_k, g = lane_k >> 4, c16 = lane_k & 15;
            // ---- recompute: E, U, A = U^+ v_x U, B = U^+ v_y U
            bool vx_in_p;
            const bool ok = wave_eigen<NP>(S, md, T0, r0, it.i0 + kk, max_iter, vx_in_p);
            if (!ok && lane == 0) atomicOr(a.status, kStatNoConv);
            v4d ar[NT][NT], ai[NT][NT], br[NT][NT], bi[NT][NT];
            {
                double2 u[NT][4][NT];
                wave_load_uops<NP>(S, u);
                if (!vx_in_p) {
                    wave_stage_velocity<NP>(S, n, md.nR0, T0, r0, true);
                    __syncthreads();
                }
                wave_rotate_mfma<NP>(S, u, ar, ai);
                __syncthreads();
                wave_stage_velocity<NP>(S, n, md.nR0, T1, r0, false);
                __syncthreads();
                wave_rotate_mfma<NP>(S, u, br, bi);
            }
            // ---- phi, phi' at the bands (lane pair per band, halves of the levels summed)
            {
                const int b = lane >> 1, h = lane & 1;
                double p = 0.0, d = 0.0;
                if (b < n) {
                    const int half = (a.nF + 1) / 2;
                    const int j0 = h * half, j1 = (h == 0) ? half : a.nF;
                    wave_phi_at(S.E[b], ef + j0, sb + j0, j1 - j0, a.kT, p, d);
                }
                p += dpp_xor1(p);
                d += dpp_xor1(d);
                if (b < n && h == 0) {
                    S.phi[b] = p;
                    S.dphi[b] = d;
                }
            }
            __syncthreads();
            // ---- K on this lane's elements
            double K[NT][NT][4];
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int tj = 0; tj < NT; ++tj)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int m = 16 * ti + g + 4 * q, c = 16 * tj + c16;
                        double kv = 0.0;
                        if (m < n && c < n && m != c) {
                            const double de = S.E[m] - S.E[c];
                            kv = (S.phi[m] - S.phi[c]) / (de * de + eta2);
                        }
                        K[ti][tj][q] = kv;
                    }
            // ---- D = (K o B) A - (K o A) B.  A operand at k-step (kt, s), row tile tr:
            // (K o B)[16 tr + c][kappa] = -K[kappa][..] conj(B[kappa][16 tr + c]) (own element)
            v4d dr[NT][NT], di[NT][NT];
#pragma unroll
            for (int x = 0; x < NT; ++x)
#pragma unroll
                for (int y = 0; y < NT; ++y) {
                    dr[x][y] = zero;
                    di[x][y] = zero;
                }
#pragma unroll
            for (int kt = 0; kt < NT; ++kt) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    double zr[NT], zi[NT], wr[NT], wi[NT];
#pragma unroll
                    for (int tr = 0; tr < NT; ++tr) {
                        const double kv = K[kt][tr][s];
                        zr[tr] = -kv * br[kt][tr][s];
                        zi[tr] = kv * bi[kt][tr][s];
                        wr[tr] = kv * ar[kt][tr][s];  // minus sign of -(K o A) folded in
                        wi[tr] = -kv * ai[kt][tr][s];
                    }
#pragma unroll
                    for (int tr = 0; tr < NT; ++tr)
#pragma unroll
                        for (int tc = 0; tc < NT; ++tc) {
                            // (z_r + i z_i)(a_r + i a_i) + (w_r + i w_i)(b_r + i b_i)
                            dr[tr][tc] = mfma16(zr[tr], ar[kt][tc][s], dr[tr][tc]);
                            di[tr][tc] = mfma16(zr[tr], ai[kt][tc][s], di[tr][tc]);
                            dr[tr][tc] = mfma16(-zi[tr], ai[kt][tc][s], dr[tr][tc]);
                            di[tr][tc] = mfma16(zi[tr], ar[kt][tc][s], di[tr][tc]);
                            dr[tr][tc] = mfma16(wr[tr], br[kt][tc][s], dr[tr][tc]);
                            di[tr][tc] = mfma16(wr[tr], bi[kt][tc][s], di[tr][tc]);
                            dr[tr][tc] = mfma16(-wi[tr], bi[kt][tc][s], dr[tr][tc]);
                            di[tr][tc] = mfma16(wi[tr], br[kt][tc][s], di[tr][tc]);
                        }
                }
            }
            // ---- X = (i/N)(D + D^+) via a transpose through S.P; Hbar' = X / (E_m - E_q)
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int tj = 0; tj < NT; ++tj)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        S.P[(16 * ti + g + 4 * q) * LD + 16 * tj + c16] = c_make(dr[ti][tj][q], di[ti][tj][q]);
            __syncthreads();
            v4d hr[NT][NT], hi[NT][NT];
            double dsum[NT][4];
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int q = 0; q < 4; ++q) dsum[ti][q] = 0.0;
            bool any_near = false;
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int tj = 0; tj < NT; ++tj)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int m = 16 * ti + g + 4 * q, c = 16 * tj + c16;
                        const double2 dt = S.P[c * LD + m];
                        double vr = 0.0, vi = 0.0;
                        if (m < n && c < n) {
                            const double de = S.E[m] - S.E[c];
                            // diagonal: Ebar_m = -(2/N) sum_p dK(E_m, E_p) Im(B_mp conj(A_mp))
                            const double x = de;
                            const double den = x * x + eta2;
                            const double w = S.dphi[m] / den - (S.phi[m] - S.phi[c]) * 2.0 * x / (den * den);
                            // (the p = m term, B_mm A_mm - A_mm B_mm, is exactly zero)
                            const double im = bi[ti][tj][q] * ar[ti][tj][q] - br[ti][tj][q] * ai[ti][tj][q];
                            if (m != c) dsum[ti][q] += w * im;
                            if (m != c) {
                                if (fabs(de) >= delta) {
                                    // (i/N)(D_mc + conj(D_cm)) / de
                                    const double sr = dr[ti][tj][q] + dt.x, si = di[ti][tj][q] - dt.y;
                                    const double f = invN / de;
                                    vr = -si * f;
                                    vi = sr * f;
                                } else {
                                    any_near = true;
                                }
                            }
                        }
                        hr[ti][tj][q] = vr;
                        hi[ti][tj][q] = vi;
                    }
            // diagonal from the row sums (the 16 lanes of a row hold its column slices)
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double tot = row16_sum(dsum[ti][q]);
                    const int m = 16 * ti + g + 4 * q;
                    if (c16 == ((g + 4 * q) & 15)) hr[ti][ti][q] = (m < n) ? -2.0 * invN * tot : 0.0;
                }
            // U operands of the back-rotations: ua[kt][s][tr] = U[16 tr + c][16 kt + g + 4 s]
            double2 ua[NT][4][NT];
#pragma unroll
            for (int kt = 0; kt < NT; ++kt)
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int tr = 0; tr < NT; ++tr) ua[kt][s][tr] = S.U[(16 * tr + c16) * LD + 16 * kt + g + 4 * s];
            __syncthreads();
            // near-degenerate pairs: the divided-difference limit, from A and B staged in LDS
            if (__ballot(any_near) != 0ull) {
#pragma unroll
                for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int idx = (16 * ti + g + 4 * q) * LD + 16 * tj + c16;
                            S.P[idx] = c_make(ar[ti][tj][q], ai[ti][tj][q]);
                            S.U[idx] = c_make(br[ti][tj][q], bi[ti][tj][q]);
                        }
                __syncthreads();
#pragma unroll
                for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int m = 16 * ti + g + 4 * q, c = 16 * tj + c16;
                            if (m < n && c < n && m != c && fabs(S.E[m] - S.E[c]) < delta) {
                                const double xm = 0.5 * (S.E[m] + S.E[c]);
                                double phx, dphx;
                                wave_phi_at(xm, ef, sb, a.nF, a.kT, phx, dphx);
                                double2 acc = c_make(0.0, 0.0);
                                for (int p = 0; p < n; ++p) {
                                    const double x = xm - S.E[p];
                                    const double den = x * x + eta2;
                                    const double w = dphx / den - (phx - S.phi[p]) * 2.0 * x / (den * den);
                                    double2 z = c_mul(S.U[m * LD + p], S.P[p * LD + c]);
                                    z = c_fnma(S.P[m * LD + p], S.U[p * LD + c], z);
                                    acc = c_add(acc, c_scale(w, z));
                                }
                                acc = c_scale(invN, c_i(acc));
                                hr[ti][tj][q] = acc.x;
                                hi[ti][tj][q] = acc.y;
                            }
                        }
                __syncthreads();
            }
            // ---- Abar = (i/N) K o B (registers); Bbar = -(i/N) K o A parked in S.U
            // (U itself is in ua now; the padding of both stays zero)
            v4d xr[NT][NT], xi[NT][NT];
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int tj = 0; tj < NT; ++tj)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double kv = invN * K[ti][tj][q];
                        xr[ti][tj][q] = -kv * bi[ti][tj][q];
                        xi[ti][tj][q] = kv * br[ti][tj][q];
                        S.U[(16 * ti + g + 4 * q) * LD + 16 * tj + c16] =
                            c_make(kv * ai[ti][tj][q], -kv * ar[ti][tj][q]);
                    }
            // ---- vbar_x = U Abar U^+, Hbar = U Hbar' U^+, vbar_y = U Bbar U^+ (all three
            // Hermitian: the upper triangle is stored for this k-point; the pencil sums
            // over the block are taken by a separate pass)
            double2* Xk = xb + it.xbuf_off + (long long)kk * 3 * nn;
            {
                v4d vr_[NT][NT], vi_[NT][NT];
                wave_sandwich<NP>(xr, xi, ua, vr_, vi_);
#pragma unroll
                for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int m = 16 * ti + g + 4 * q, c = 16 * tj + c16;
                            if (m <= c && c < n) Xk[nn + (long long)m * n + c] = c_make(vr_[ti][tj][q], vi_[ti][tj][q]);
                        }
            }
            {
                v4d hbr[NT][NT], hbi[NT][NT];
                wave_sandwich<NP>(hr, hi, ua, hbr, hbi);
#pragma unroll
                for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int m = 16 * ti + g + 4 * q, c = 16 * tj + c16;
                            if (m <= c && c < n) Xk[(long long)m * n + c] = c_make(hbr[ti][tj][q], hbi[ti][tj][q]);
                        }
            }
            {
                v4d yr[NT][NT], yi[NT][NT];
#pragma unroll
                for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const double2 v = S.U[(16 * ti + g + 4 * q) * LD + 16 * tj + c16];
                            yr[ti][tj][q] = v.x;
                            yi[ti][tj][q] = v.y;
                        }
                v4d vyr[NT][NT], vyi[NT][NT];
                wave_sandwich<NP>(yr, yi, ua, vyr, vyi);
#pragma unroll
                for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int m = 16 * ti + g + 4 * q, c = 16 * tj + c16;
                            if (m <= c && c < n) Xk[2 * nn + (long long)m * n + c] = c_make(vyr[ti][tj][q], vyi[ti][tj][q]);
                        }
            }
            __syncthreads();
        }
    }
}

template <int NP>
static hipError_t launch_adjoint_wave_t(const WgLaunch& L, hipStream_t s) {
    const size_t lds = sizeof(WaveLds<NP>);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_adjoint_wave<NP>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int units = L.item_count * L.unit_parts;
    const int grid = units < L.max_groups ? units : L.max_groups;
    hipLaunchKernelGGL((k_adjoint_wave<NP>), dim3(grid), dim3(64), lds, s, L);
    return hipGetLastError();
}

hipError_t launch_adjoint_wave(const WgLaunch& L, int np, hipStream_t s) {
    if (L.item_count <= 0) return hipSuccess;
    if (!L.queue || L.unit_k < 1 || L.unit_parts < 1) return hipErrorInvalidValue;
    if (np <= 16) return launch_adjoint_wave_t<16>(L, s);
    if (np <= 32) return launch_adjoint_wave_t<32>(L, s);
    return hipErrorInvalidValue;
}

}  // namespace kubo
