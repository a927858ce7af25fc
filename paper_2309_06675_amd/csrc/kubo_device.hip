// kubo_device.hip -- gfx950 kernels of the Kubo-formula Hall-conductivity path.
//
// Forward pipeline for one batch of k-points (paper: the four per-k steps of
// the baseline listing, batched as in its Eq. (4)):
//   k_hermproj   t'(R) = (t(R) + t(-R)^+)/2, so that H(k) = sum_R t'(R) e^{ik.R}
//                is the Hermitian part of the Bloch sum.
//   k_pencil     sum factorisation of the Bloch sum over one kx pencil:
//                T_rho  = sum_{R: R_x = rho} t'(R) e^{i(k1 R_y + k2 R_z)}
//                Ty_rho = sum_{R: R_x = rho} i R_y t'(R) e^{i(k1 R_y + k2 R_z)}
//                (and, for the Hall tensor, Tz_rho with i R_z likewise)
//   per-k kernels (kubo_wave.hip for n <= 32, kubo_wg.hip for larger n and for
//                the adjoint): H = sum_rho e^{i k0 rho} T_rho,
//                v_x = sum_rho i rho e^{i k0 rho} T_rho, v_y = sum_rho e^{i k0 rho} Ty_rho
//                (step 1); Hermitian eigendecomposition (step 2); A = U^+ v_x U,
//                B = U^+ v_y U (step 3); Berry curvature
//                Omega_n = -2 sum_m Im(A_nm B_mn) g(E_n - E_m) and the Fermi-weighted
//                sums s_j = sum_n f_j(E_n) Omega_n accumulated per k-block (step 4).
//   k_reduce     sigma_j = -(1/N_k) sum over the model's k-blocks, fixed tree order.
// The Hall tensor variant of the per-k kernels also rotates v_z and the spin
// current into the eigenbasis and accumulates four components per level.
//   k_gacc, k_gsym  the adjoint's transposed Bloch sum and Hermitian-projection rule.
// All arithmetic is FP64.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kubo_cplx.h"
#include "kubo_internal.h"
#include "kubo_launch.h"

namespace kubo {

// ---------------------------------------------------------------------------
// k_clear: zero the status word (a kernel, not a memset, so graphs replay it)
// ---------------------------------------------------------------------------
__global__ void k_clear_status(unsigned* status, unsigned* queues, int n_queue_words) {
    if (threadIdx.x == 0) status[0] = 0u;
    for (int i = threadIdx.x; i < n_queue_words; i += blockDim.x) queues[i] = 0u;
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
// k_pencil: per (model, i1, i2) the rho-resolved partial Bloch sums, for a group
// of up to kPencilGroup pencils of one model and one k_z index (i2) at a time.
// Each thread owns one matrix element.  The lattice vectors of an R_x group come
// ordered by (R_y, R_z), so each run of equal R_y is first summed over R_z with
// the group's common k_z phase, reading each hopping t'(R) once, and the run's sum
// then goes into every pencil of the group with that pencil's k_y phase (the sum
// over R factorised as sum over R_y of e^{i k_y R_y} sum over R_z).  Phases sit in
// LDS, a tile of lattice vectors at a time.  Grid: x = pencil group, y = tile of
// 256 matrix elements.
// ---------------------------------------------------------------------------
constexpr int kPencilThreads = 256;
constexpr int kPencilPhaseTile = 256;

__global__ __launch_bounds__(kPencilThreads) void k_pencil(Tables tb, int group_begin,
                                                           const double2* __restrict__ tp,
                                                           double2* __restrict__ tbuf, bool with_z) {
    __shared__ double2 sph[kPencilPhaseTile][kPencilGroup];  // e^{i k_y(q) R_y(g)}
    __shared__ double2 sphz[kPencilPhaseTile];               // e^{i k_z R_z(g)}
    const PencilGroup grp = tb.pgroups[group_begin + blockIdx.x];
    const PencilItem p0 = tb.pencils[grp.first];
    const ModelDev md = tb.models[p0.model];
    const int n = md.n;
    const long long nn = (long long)n * n;
    if ((long long)blockIdx.y * kPencilThreads >= nn) return;  // whole workgroup past the matrix
    const long long e = (long long)blockIdx.y * kPencilThreads + threadIdx.x;
    const bool act = e < nn;
    const int cnt = grp.count;
    const int* gstart = tb.grp_start + md.gs_first;
    for (int rho = 0; rho < md.nR0; ++rho) {
        const int g0 = gstart[rho], g1 = gstart[rho + 1];
        double2 a0[kPencilGroup], a1[kPencilGroup], a2[kPencilGroup];
#pragma unroll
        for (int q = 0; q < kPencilGroup; ++q) a0[q] = a1[q] = a2[q] = c_make(0.0, 0.0);
        for (int gt = g0; gt < g1; gt += kPencilPhaseTile) {
            const int gcount = min(kPencilPhaseTile, g1 - gt);
            __syncthreads();
            for (int idx = threadIdx.x; idx < gcount * (kPencilGroup + 1); idx += kPencilThreads) {
                const int g = idx / (kPencilGroup + 1), q = idx - g * (kPencilGroup + 1);
                const int gi = md.grp_first + gt + g;
                if (q == kPencilGroup) {
                    sphz[g] = unit_phase((long long)p0.i2 * tb.grp_R2[gi], md.N2);
                } else {
                    double2 ph = c_make(0.0, 0.0);
                    if (q < cnt) ph = unit_phase((long long)tb.pencils[grp.first + q].i1 * tb.grp_R1[gi], md.N1);
                    sph[g][q] = ph;
                }
            }
            __syncthreads();
            if (act) {
                // the current run of equal R_y: its R_z sums (u; uz for v_z) and the tile
                // index of its first lattice vector (whose k_y phases the run takes)
                double2 u = c_make(0.0, 0.0), uz = u;
                int run_g = -1, run_ry = 0;
                auto flush = [&]() {
                    const double2 uy = c_i(c_scale((double)run_ry, u));
#pragma unroll
                    for (int q = 0; q < kPencilGroup; ++q) {
                        if (q < cnt) {
                            const double2 py = sph[run_g][q];
                            a0[q] = c_fma(u, py, a0[q]);
                            a1[q] = c_fma(uy, py, a1[q]);
                            if (with_z) a2[q] = c_fma(uz, py, a2[q]);
                        }
                    }
                };
                for (int g = 0; g < gcount; ++g) {
                    const int gi = md.grp_first + gt + g;
                    const int ry = tb.grp_R1[gi];
                    if (run_g < 0 || ry != run_ry) {
                        if (run_g >= 0) flush();
                        u = uz = c_make(0.0, 0.0);
                        run_g = g;
                        run_ry = ry;
                    }
                    const double2 v = tp[md.t_off + (long long)tb.grp_r[gi] * nn + e];
                    const double2 pz = sphz[g];
                    u = c_fma(v, pz, u);
                    if (with_z) uz = c_fma(c_i(c_scale((double)tb.grp_R2[gi], v)), pz, uz);
                }
                if (run_g >= 0) flush();  // a run that goes on in the next tile restarts there
            }
        }
        if (act) {
#pragma unroll
            for (int q = 0; q < kPencilGroup; ++q) {
                if (q < cnt) {
                    double2* T0 = tbuf + tb.pencils[grp.first + q].tbuf_off;
                    T0[(long long)rho * nn + e] = a0[q];
                    T0[(long long)(md.nR0 + rho) * nn + e] = a1[q];
                    if (with_z) T0[(long long)(2 * md.nR0 + rho) * nn + e] = a2[q];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// k_gacc: grad_t(R) += sum_{blocks} e^{-i(k1 R_y + k2 R_z)} (PH_rho - i R_y PY_rho), rho = R_x,
// for one range of k-blocks of one model (fixed order over the blocks).
// Grid: x = lattice vector in grouped order, y = tile of matrix entries, z = range.
// ---------------------------------------------------------------------------
constexpr int kGaccThreads = 128;
constexpr int kGaccRB = 4;      // lattice vectors of one R_x group per workgroup
constexpr int kGaccBlocks = 64; // k-blocks whose phases sit in LDS at a time

// G(R) += sum_blocks e^{-i(k1 R_y + k2 R_z)} (PH_rho - i R_y PY_rho) for a batch of up to
// kGaccRB lattice vectors sharing R_x = rho: each block's PH_rho, PY_rho element is read
// once and serves the whole batch (small batches and element tiles keep enough
// workgroups in flight).  Grid: (rho, batch) x element tiles x block ranges.
__global__ __launch_bounds__(kGaccThreads) void k_gacc(Tables tb, const GaccRange* __restrict__ ranges,
                                                       int range_begin, int nbatch,
                                                       const double2* __restrict__ pbuf,
                                                       double2* __restrict__ grad) {
    __shared__ double2 sph[kGaccRB][kGaccBlocks];
    __shared__ long long soff[kGaccBlocks];
    const GaccRange rg = ranges[range_begin + blockIdx.z];
    const ModelDev md = tb.models[rg.model];
    const int rho = (int)blockIdx.x / nbatch, batch = (int)blockIdx.x - rho * nbatch;
    if (rho >= md.nR0) return;
    const int* gs = tb.grp_start + md.gs_first;
    const int g0 = gs[rho] + batch * kGaccRB;
    const int g1 = min(gs[rho + 1], g0 + kGaccRB);
    if (g0 >= g1) return;
    const int nb = g1 - g0;
    const int n = md.n;
    const long long nn = (long long)n * n;
    if ((long long)blockIdx.y * kGaccThreads >= nn) return;
    const long long e = (long long)blockIdx.y * kGaccThreads + threadIdx.x;
    int R1[kGaccRB];
#pragma unroll
    for (int q = 0; q < kGaccRB; ++q) R1[q] = (q < nb) ? tb.grp_R1[md.grp_first + g0 + q] : 0;
    double2 acc[kGaccRB];
#pragma unroll
    for (int q = 0; q < kGaccRB; ++q) acc[q] = c_make(0.0, 0.0);
    for (int b0 = 0; b0 < rg.count; b0 += kGaccBlocks) {
        const int bc = min(kGaccBlocks, rg.count - b0);
        __syncthreads();
        for (int idx = threadIdx.x; idx < bc * nb; idx += kGaccThreads) {
            const int q = idx / bc, b = idx - q * bc;
            const BlockItem bi = tb.blocks[rg.begin + b0 + b];
            const int gi = md.grp_first + g0 + q;
            sph[q][b] = unit_phase2(-(long long)bi.i1 * tb.grp_R1[gi], md.N1,
                                    -(long long)bi.i2 * tb.grp_R2[gi], md.N2);
            if (q == 0) soff[b] = bi.pbuf_off;
        }
        __syncthreads();
        if (e < nn) {
#pragma unroll 4
            for (int b = 0; b < bc; ++b) {
                const double2* P = pbuf + soff[b];
                const double2 h = P[(long long)rho * nn + e];
                const double2 y = P[(long long)(md.nR0 + rho) * nn + e];
#pragma unroll
                for (int q = 0; q < kGaccRB; ++q) {
                    if (q < nb) {
                        const double2 w = c_sub(h, c_scale((double)R1[q], c_i(y)));
                        acc[q] = c_fma(sph[q][b], w, acc[q]);
                    }
                }
            }
        }
    }
    if (e < nn) {
#pragma unroll
        for (int q = 0; q < kGaccRB; ++q) {
            if (q < nb) {
                const int r = tb.grp_r[md.grp_first + g0 + q];
                double2* G = grad + md.t_off + (long long)r * nn + e;
                *G = c_add(*G, acc[q]);
            }
        }
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
__global__ __launch_bounds__(kReduceThreads) void k_reduce(Tables tb, int nF, int ncomp,
                                                           const double* __restrict__ partial,
                                                           double* __restrict__ sigma,
                                                           unsigned* status) {
    __shared__ double red[kReduceThreads];
    const int m = blockIdx.y;
    const int j = blockIdx.x;
    const ModelDev md = tb.models[m];
    double s = 0.0;
    const int w = nF * ncomp;  // j runs over the components' levels, [ncomp][nF]
    for (int k = threadIdx.x; k < md.slot_count; k += kReduceThreads)
        s += partial[(long long)(md.slot_first + k) * w + j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double v = -red[0] / (double)md.Nk;
        if (!isfinite(v)) atomicOr(status, kStatNonFinite);
        sigma[(long long)md.f_off * ncomp + j] = v;
    }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
hipError_t launch_clear(unsigned* status, unsigned* queues, int n_queue_words, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(256), 0, s, status, queues, n_queue_words);
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

// ---------------------------------------------------------------------------
// k_pacc: pencil sums of the one-wavefront adjoint's per-k matrices (Hermitian,
// upper triangle stored; the lower one is read as the conjugate transpose), one
// workgroup per (k-block, 256 matrix elements).  For each R_x value rho:
//   PH_rho = sum_k e^{-i k0 rho} (Hbar - i rho vbar_x),  PY_rho = sum_k e^{-i k0 rho} vbar_y,
// summed over the block's k-points in order.  The phases of up to 32
// k-points at a time sit in LDS.
// ---------------------------------------------------------------------------
constexpr int kPaccThreads = 256;
constexpr int kPaccTile = 32;

__global__ __launch_bounds__(kPaccThreads) void k_pacc(Tables tb, int begin, const double2* __restrict__ xbuf,
                                                        double2* __restrict__ pbuf, unsigned* status) {
    __shared__ double2 ph[kPaccTile][kMaxR0];
    const BlockItem it = tb.blocks[begin + blockIdx.x];
    const ModelDev md = tb.models[it.model];
    const long long nn = (long long)md.n * md.n;
    if ((long long)blockIdx.y * kPaccThreads >= nn) return;  // whole workgroup past this matrix
    const long long e = (long long)blockIdx.y * kPaccThreads + threadIdx.x;
    const bool act = e < nn;
    // the per-k matrices are Hermitian: stored whole (xfull) or as their upper triangle
    const int em = act ? (int)(e / md.n) : 0, ec = act ? (int)(e - (long long)em * md.n) : 0;
    const bool lower = !it.xfull && em > ec;
    const long long es = lower ? (long long)ec * md.n + em : e;
    const int nR0 = md.nR0;
    const int* r0 = tb.r0val + md.r0_first;
    const double2* X = xbuf + it.xbuf_off;
    double2 accH[kMaxR0], accY[kMaxR0];
#pragma unroll
    for (int rho = 0; rho < kMaxR0; ++rho) {
        accH[rho] = c_make(0.0, 0.0);
        accY[rho] = c_make(0.0, 0.0);
    }
    for (int k0 = 0; k0 < it.count; k0 += kPaccTile) {
        const int kc = (it.count - k0 < kPaccTile) ? it.count - k0 : kPaccTile;
        __syncthreads();
        for (int idx = threadIdx.x; idx < kc * nR0; idx += kPaccThreads) {
            const int kk = idx / nR0, rho = idx - kk * nR0;
            ph[kk][rho] = c_conj(unit_phase((long long)(it.i0 + k0 + kk) * r0[rho], md.N0));
        }
        __syncthreads();
        if (act) {
            for (int kk = 0; kk < kc; ++kk) {
                const double2* Xk = X + (long long)(k0 + kk) * 3 * nn;
                double2 h = Xk[es], vx = Xk[nn + es], vy = Xk[2 * nn + es];
                if (lower) {
                    h = c_conj(h);
                    vx = c_conj(vx);
                    vy = c_conj(vy);
                }
                const bool first = (k0 + kk == 0);
#pragma unroll
                for (int rho = 0; rho < kMaxR0; ++rho) {
                    if (rho < nR0) {
                        const double2 pc = ph[kk][rho];
                        const double rr = (double)r0[rho];
                        const double2 w = c_make(h.x + rr * vx.y, h.y - rr * vx.x);
                        const double2 h1 = c_mul(pc, w);
                        const double2 y1 = c_mul(pc, vy);
                        accH[rho] = first ? h1 : c_add(accH[rho], h1);
                        accY[rho] = first ? y1 : c_add(accY[rho], y1);
                    }
                }
            }
        }
    }
    if (act) {
        double2* PH = pbuf + it.pbuf_off;
        double2* PY = PH + (long long)nR0 * nn;
        bool bad = false;
#pragma unroll
        for (int rho = 0; rho < kMaxR0; ++rho) {
            if (rho < nR0) {
                PH[rho * nn + e] = accH[rho];
                PY[rho * nn + e] = accY[rho];
                bad |= !isfinite(accH[rho].x + accH[rho].y + accY[rho].x + accY[rho].y);
            }
        }
        if (bad) atomicOr(status, kStatNonFinite);
    }
}

hipError_t launch_pencil(const Tables& tb, int group_begin, int group_count, long long max_nn,
                         const double* tp, double* tbuf, bool with_z, hipStream_t s) {
    if (group_count <= 0) return hipSuccess;
    const unsigned ty = (unsigned)((max_nn + kPencilThreads - 1) / kPencilThreads);
    hipLaunchKernelGGL(k_pencil, dim3(group_count, ty), dim3(kPencilThreads), 0, s, tb, group_begin,
                       reinterpret_cast<const double2*>(tp), reinterpret_cast<double2*>(tbuf),
                       with_z);
    return hipGetLastError();
}

hipError_t launch_pacc(const Tables& tb, int begin, int count, long long max_nn, const double* xbuf,
                       double* pbuf, unsigned* status, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const unsigned ty = (unsigned)((max_nn + kPaccThreads - 1) / kPaccThreads);
    hipLaunchKernelGGL(k_pacc, dim3(count, ty), dim3(kPaccThreads), 0, s, tb, begin,
                       reinterpret_cast<const double2*>(xbuf), reinterpret_cast<double2*>(pbuf), status);
    return hipGetLastError();
}

hipError_t launch_gacc(const Tables& tb, const GaccRange* ranges, int range_begin, int range_count,
                       int max_group, long long max_nn, const double* pbuf, double* grad,
                       hipStream_t s) {
    if (range_count <= 0) return hipSuccess;
    const int nbatch = (max_group + kGaccRB - 1) / kGaccRB;
    const unsigned ty = (unsigned)((max_nn + kGaccThreads - 1) / kGaccThreads);
    hipLaunchKernelGGL(k_gacc, dim3(kMaxR0 * nbatch, ty, range_count), dim3(kGaccThreads), 0, s, tb,
                       ranges, range_begin, nbatch, reinterpret_cast<const double2*>(pbuf),
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

hipError_t launch_reduce(const Tables& tb, int n_models, int nF, int ncomp, const double* partial,
                         double* sigma, unsigned* status, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(nF * ncomp, n_models), dim3(kReduceThreads), 0, s, tb, nF,
                       ncomp, partial, sigma, status);
    return hipGetLastError();
}

}  // namespace kubo
