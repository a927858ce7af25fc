// kubo_cplx.h -- device helpers shared by the HIP kernels: complex FP64
// arithmetic on double2 (x = re, y = im), exact-angle unit phases and the
// occupation function.
#pragma once

#include <hip/hip_runtime.h>

namespace kubo {

// ---------------------------------------------------------------------------
// complex helpers (double2: x = re, y = im)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 c_make(double r, double i) { return make_double2(r, i); }
__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return c_make(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return c_make(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 c_conj(double2 a) { return c_make(a.x, -a.y); }
__device__ __forceinline__ double2 c_scale(double s, double2 a) { return c_make(s * a.x, s * a.y); }
__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
    return c_make(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// acc + a * b
__device__ __forceinline__ double2 c_fma(double2 a, double2 b, double2 acc) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
// acc - a * b
__device__ __forceinline__ double2 c_fnma(double2 a, double2 b, double2 acc) {
    acc.x = fma(-a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(-a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}
// acc + conj(a) * b
__device__ __forceinline__ double2 c_fmac(double2 a, double2 b, double2 acc) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}
// i * a
__device__ __forceinline__ double2 c_i(double2 a) { return c_make(-a.y, a.x); }

// e^{2 pi i m / N} for an integer residue m (reduced to (-N/2, N/2] first).
__device__ __forceinline__ double2 unit_phase(long long m, long long N) {
    m %= N;
    if (m < 0) m += N;
    if (2 * m > N) m -= N;
    // separate sine and cosine: sincospi returns its cosine through private memory
    const double x = 2.0 * (double)m / (double)N;
    return c_make(cospi(x), sinpi(x));
}

// e^{i (2 pi a1/N1 + 2 pi a2/N2)} with exact rational reduction of the angle.
__device__ __forceinline__ double2 unit_phase2(long long a1, long long N1, long long a2,
                                               long long N2) {
    long long m1 = a1 % N1, m2 = a2 % N2;
    return unit_phase(m1 * N2 + m2 * N1, N1 * N2);
}

// Occupation: Fermi-Dirac at kT > 0, a step with f(E_F) = 1/2 at kT = 0.
// One exponential of -|u| serves both signs (no divergent branch), and the
// quotient uses a Newton-refined reciprocal.
__device__ __forceinline__ double occupation(double e, double ef, double kT) {
    if (kT == 0.0) return e < ef ? 1.0 : (e > ef ? 0.0 : 0.5);
    const double u = (e - ef) / kT;
    const double w = exp(-fabs(u));
    const double d = 1.0 + w;
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    return (u > 0.0) ? w * r : r;
}

// The same with 1/kT supplied (a multiplication instead of a division per call).
__device__ __forceinline__ double occupation_ikt(double e, double ef, double kT, double ikT) {
    if (kT == 0.0) return e < ef ? 1.0 : (e > ef ? 0.0 : 0.5);
    const double u = (e - ef) * ikT;
    const double w = exp(-fabs(u));
    const double d = 1.0 + w;
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    return (u > 0.0) ? w * r : r;
}

// conj(a) * b  and  a * conj(b)
__device__ __forceinline__ double2 c_cmul(double2 a, double2 b) {
    return c_make(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 c_mulc(double2 a, double2 b) {
    return c_make(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// acc - a conj(b) - c conj(d) (a Hermitian rank-2 update) as eight chained FMAs
__device__ __forceinline__ double2 c_rank2c(double2 acc, double2 a, double2 b, double2 c, double2 d) {
    acc.x = fma(-a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.x = fma(-c.x, d.x, acc.x);
    acc.x = fma(-c.y, d.y, acc.x);
    acc.y = fma(-a.y, b.x, acc.y);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-c.y, d.x, acc.y);
    acc.y = fma(c.x, d.y, acc.y);
    return acc;
}

// Work queue of the persistent per-k kernels.  A launch's work units are split
// into eight equal bins, one per XCD: workgroups are handed to the XCDs
// round-robin (workgroup b runs on XCD b % 8), so the consecutive units of a bin
// (the k-blocks of one pencil, which read the same partial Bloch sums) run inside
// one XCD and share its L2.  A workgroup takes the next unit of its own bin with
// an atomic counter (ctr[0..7], zero at the start of the launch) and, once that
// bin is empty, the next units of the other bins in turn, so units of uneven cost
// balance over the whole GPU and no XCD idles while another has work.  Returns -1
// when every bin is empty (then every later call returns -1 too).  Called by one
// lane; `probe` is that lane's state (0 before the first call).
__device__ __forceinline__ int queue_take(unsigned* ctr, int count, int& probe) {
    const int x = (int)blockIdx.x & 7;
    while (probe < 8) {
        const int b = (x + probe) & 7;
        const int lo = (int)((long long)count * b / 8), hi = (int)((long long)count * (b + 1) / 8);
        if (lo < hi) {
            const unsigned i = atomicAdd(ctr + b, 1u);
            if (i < (unsigned)(hi - lo)) return lo + (int)i;
        }
        ++probe;
    }
    return -1;
}

}  // namespace kubo
