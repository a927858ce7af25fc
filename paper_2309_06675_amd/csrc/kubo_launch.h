// kubo_launch.h -- host-callable launchers of the device kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/kubo.h"
#include "kubo_internal.h"

namespace kubo {

struct FwdLaunch {
    Tables tb;
    const double* tbuf;
    const double* e_fermi;
    double* partial;
    unsigned* status;
    double eta, kT;
    int nF;
    int max_sweeps;
    int item_begin, item_count;
    int np;          // padded size class of every item in the list
    int max_groups;  // persistent grid size cap
    // Hall tensor (tensor != 0): the pencil partials hold a third set (the i R_z sums), the
    // partial sums four components per slot ([slot][4][nF]: xy, yz, zx, spin Hall), and
    // spin (per orbital, all models; NULL: no spin Hall component) weights the spin current
    int tensor;
    const double* spin;
    unsigned* queue;  // this launch's eight work-queue counters, zero at its start
};

struct WgLaunch {
    Tables tb;
    const double* tbuf;
    double* pbuf;
    const double* e_fermi;
    const double* sbar;
    double* partial;
    unsigned* status;
    double* scratch;       // max_groups slots of slot_elems complex elements
    double* xbuf;          // per-k adjoint matrices of the one-wavefront classes
    long long slot_elems;
    double eta, kT;
    int nF;
    int max_iter;
    int item_begin, item_count;
    int max_groups;
    int tensor;           // forward only: as FwdLaunch::tensor
    const double* spin;   // forward only: as FwdLaunch::spin
    unsigned* queue;      // this launch's eight work-queue counters, zero at its start
    // work unit u covers k-points [p*unit_k, (p+1)*unit_k) of item u / unit_parts,
    // p = u % unit_parts (the forward: unit_parts = 1, one unit per item)
    int unit_k, unit_parts;
};

// The Green's-function form (n <= 32): one workgroup per k-point, every item of
// the list has n <= 32 whatever its size class.
struct GfLaunch {
    Tables tb;
    const double* tbuf;
    const double* e_fermi;
    const double* omega;   // [n_omega] nodes of the half-line quadrature (device)
    const double* weight;  // [n_omega] its weights (device)
    double* partial;       // [slot][nF]
    unsigned* status;
    unsigned* queue;       // this launch's eight work-queue counters, zero at its start
    double gamma;
    int nF, n_omega;
    int item_begin, item_count;
    int max_groups;
};
hipError_t launch_gf(const GfLaunch& L, hipStream_t s);

// The large-n path (kBigMinN < n <= kBigMaxN): a batch of `count` items (one
// k-point each) of one model of size n, each with a workspace slice of per_k
// complex elements laid out by big_layout.
constexpr int kBigMaxN = 512;
constexpr int kBigB = 32;          // reflectors per compact-WY block
constexpr double kBigGap = 1e-5;   // relative gap below which eigenvalues form a cluster
constexpr int kBigBatch = 256;     // most k-points of one pipeline pass
struct BigLayout {
    long long H, VX, VY, U, X, V, W, W2, TF, tau;  // complex offsets
    long long d, e, E, piv, blk;                   // double offsets (from the start of the slice)
    long long per_k;                               // complex elements per k-point
};
__host__ __device__ inline BigLayout big_layout(int n) {
    const long long nn = (long long)n * n;
    const long long nb = (n + kBigB - 1) / kBigB;
    BigLayout L;
    L.H = 0;
    L.VX = L.H + nn;
    L.VY = L.VX + nn;
    L.U = L.VY + nn;
    L.X = L.U + nn;
    L.V = L.X + nn;
    L.W = L.V + nn;
    L.W2 = L.W + (long long)kBigB * n;
    L.TF = L.W2 + (long long)kBigB * n;
    L.tau = L.TF + nb * kBigB * kBigB;
    const long long dbase = 2 * (L.tau + n);  // doubles
    L.d = dbase;
    L.e = L.d + n;
    L.E = L.e + n;
    L.piv = L.E + n;          // 6 n doubles per eigenvalue thread
    L.blk = L.piv + 6 * nn;   // n ints (stored in n doubles)
    L.per_k = (L.blk + n + 1) / 2 + 1;
    return L;
}
struct BigLaunch {
    Tables tb;
    const double* tbuf;
    const double* e_fermi;
    double* partial;
    unsigned* status;
    double* scratch;  // count slices of per_k complex elements
    long long per_k;
    double eta, kT;
    int nF;
    int n;
    int item_begin, count;
};
struct BigGemm {
    const double2* A;
    const double2* B;
    double2* C;
    long long sa, sb, sc;  // batch strides (complex elements)
    int lda, ldb, ldc;
    int M, N, K;
    double alpha;
    int beta;
};
// red_start / red_stop (null: none): events recorded around the reduction kernel
hipError_t launch_big_forward(const BigLaunch& L, hipStream_t s, hipEvent_t red_start = nullptr,
                              hipEvent_t red_stop = nullptr);

long long wg_slot_elems(int nmax);
// np: the size class (64: n <= 64, 128: n <= 128)
hipError_t launch_forward_wg(const WgLaunch& L, int np, hipStream_t s);
hipError_t launch_adjoint_wg(const WgLaunch& L, int np, hipStream_t s);
// one wavefront per k-point for n <= 32 (np: the size class, 8, 16 or 32)
hipError_t launch_adjoint_wave(const WgLaunch& L, int np, hipStream_t s);

// zero the status word and n_queue_words work-queue counters (a kernel, so that it
// is also a plain kernel node when captured into a graph)
hipError_t launch_clear(unsigned* status, unsigned* queues, int n_queue_words, hipStream_t s);
hipError_t launch_zero(double* p, long long count, hipStream_t s);
hipError_t launch_hermproj(const Tables& tb, int n_models, long long total, const double* t,
                           double* tp, hipStream_t s);
// the partial Bloch sums of the pencil groups [group_begin, group_begin + group_count);
// with_z: also the i R_z-weighted sums (third set, for the Hall tensor)
hipError_t launch_pencil(const Tables& tb, int group_begin, int group_count, long long max_nn,
                         const double* tp, double* tbuf, bool with_z, hipStream_t s);
hipError_t launch_forward_wave(const FwdLaunch& L, hipStream_t s);
// pencil sums of the adjoint matrices of blocks [begin, begin + count):
// PH_rho = sum_k e^{-i k0 rho}(Hbar - i rho vbar_x), PY_rho = sum_k e^{-i k0 rho} vbar_y
hipError_t launch_pacc(const Tables& tb, int begin, int count, long long max_nn, const double* xbuf,
                       double* pbuf, unsigned* status, hipStream_t s);
// max_group: the largest number of lattice vectors sharing one R_x value
hipError_t launch_gacc(const Tables& tb, const GaccRange* ranges, int range_begin, int range_count,
                       int max_group, long long max_nn, const double* pbuf, double* grad,
                       hipStream_t s);
hipError_t launch_gsym(const Tables& tb, int n_models, long long total, double* grad,
                       hipStream_t s);
// ncomp components per slot and per model: partial [slot][ncomp * nF], sigma
// [model][ncomp * nF]
hipError_t launch_reduce(const Tables& tb, int n_models, int nF, int ncomp, const double* partial,
                         double* sigma, unsigned* status, hipStream_t s);

// The body of kubo_ahc on a given workspace.  allow_graph = false: eager
// launches only, and no timing events (the no-allocation entry point).
kubo_status ahc_enqueue(kubo_plan_t plan, const double* t, const double* e_fermi, double eta,
                        double kT, double* sigma, void* workspace, size_t workspace_bytes,
                        void* stream, bool allow_graph, bool tensor = false,
                        const double* spin = nullptr);

}  // namespace kubo
