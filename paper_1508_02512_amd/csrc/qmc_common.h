// Device helpers shared by the real and complex integrand kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "qmc_device.h"

namespace qmc {

// Inputs that no kernel writes (sector headers, lattices, term tables,
// shifts, work items) are read through the constant address space: the
// compiler may then fetch wave-uniform values with scalar loads into SGPRs
// instead of vector loads into VGPRs, which it must otherwise assume the
// kernel's own stores could alias.
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

template <typename T>
__device__ __forceinline__ cptr<T> ro(const T *p)
{
    return (cptr<T>)p;
}

// one work item, field by field (a struct copy out of the constant address
// space is not expressible)
__device__ __forceinline__ qmc_item load_item(const qmc_item *items, int i)
{
    cptr<qmc_item> p = ro(items) + i;
    qmc_item it;
    it.sector = p->sector;
    it.point = p->point;
    it.shift = p->shift;
    it.group = p->group;
    it.lat = p->lat;
    it.start = p->start;
    it.count = p->count;
    it.stride = p->stride;
    return it;
}

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ void neumaier(double &s, double &c, double x)
{
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
    s = t;
}

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Korobov periodiser of order r: t = psi_r(y), 1 - t = psi_r(1 - y), weight
// w = y^r (1-y)^r / B(r+1, r+1).  r = 1 is Eq. 21 (3y^2 - 2y^3).
__device__ __forceinline__ void korobov(int r, double y, double &t, double &omt,
                                        double &w)
{
    const double u = 1.0 - y;
    if (r == 2) {
        t = y * y * y * fma(y, fma(6.0, y, -15.0), 10.0);
        omt = u * u * u * fma(u, fma(6.0, u, -15.0), 10.0);
        w = 30.0 * (y * u) * (y * u);
    } else if (r == 1) {
        t = y * y * fma(-2.0, y, 3.0);
        omt = u * u * fma(-2.0, u, 3.0);
        w = 6.0 * y * u;
    } else if (r == 3) {
        t = y * y * y * y * fma(y, fma(y, fma(-20.0, y, 70.0), -84.0), 35.0);
        omt = u * u * u * u * fma(u, fma(u, fma(-20.0, u, 70.0), -84.0), 35.0);
        const double yu = y * u;
        w = 140.0 * yu * yu * yu;
    } else {
        t = y;
        omt = u;
        w = 1.0;
    }
}

// prod_j t_j^e_j for exponents packed 4 bits per variable (wave-uniform)
__device__ __forceinline__ double monomial(uint32_t e, const double *t,
                                           const double *t2, const double *t3)
{
    double v = 1.0;
#pragma unroll
    for (int j = 0; j < QMC_DMAX; ++j) {
        const uint32_t ej = (e >> (4 * j)) & 15u;
        if (ej == 0u) continue;
        if (ej == 1u) {
            v *= t[j];
        } else if (ej == 2u) {
            v *= t2[j];
        } else if (ej == 3u) {
            v *= t3[j];
        } else {
            double p = t2[j] * t2[j];
            for (uint32_t k = 4u; k < ej; ++k) p *= t[j];
            v *= p;
        }
    }
    return v;
}

__device__ __forceinline__ double ipow(double x, int e)
{
    // e is wave-uniform; negative powers by one division
    double r = 1.0;
    const int a = e < 0 ? -e : e;
    for (int k = 0; k < a; ++k) r *= x;
    return e < 0 ? 1.0 / r : r;
}

// --------------------------------------------------------- block reduce

template <int K, int NC>
__device__ __forceinline__ void block_reduce_store(double (&s)[NC][K], double (&c)[NC][K],
                                                   double *dst, int kstride)
{
    __shared__ double red[QMC_BLOCK / 64][NC][K][2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int p = 0; p < NC; ++p) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            double ss = s[p][q], cc = c[p][q];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double os = __shfl_xor(ss, off);
                const double oc = __shfl_xor(cc, off);
                double e;
                two_sum(ss, os, ss, e);
                cc = cc + oc + e;
            }
            if (lane == 0) {
                red[wave][p][q][0] = ss;
                red[wave][p][q][1] = cc;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < kstride) {
        const int q = threadIdx.x;
        if (q < K) {
#pragma unroll
            for (int p = 0; p < NC; ++p) {
                double ss = red[0][p][q][0], cc = red[0][p][q][1];
#pragma unroll
                for (int w = 1; w < QMC_BLOCK / 64; ++w) {
                    double e;
                    two_sum(ss, red[w][p][q][0], ss, e);
                    cc = cc + red[w][p][q][1] + e;
                }
                dst[(size_t)q * 4 + 2 * p] = ss;
                dst[(size_t)q * 4 + 2 * p + 1] = cc;
            }
            if (NC == 1) {
                dst[(size_t)q * 4 + 2] = 0.0;
                dst[(size_t)q * 4 + 3] = 0.0;
            }
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) dst[(size_t)q * 4 + c] = 0.0;
        }
    }
}

__device__ __forceinline__ void store_violations(int viol, int32_t *dst)
{
    __shared__ int vsum;
    if (threadIdx.x == 0) vsum = 0;
    __syncthreads();
    if (viol) atomicAdd(&vsum, viol);
    __syncthreads();
    if (threadIdx.x == 0) *dst = vsum;
}

// Product of the four power-table factors a term program word lists
// (slots 2 j: t_j, 2 j + 1: t_j^2, 16: 1), read from this lane's column of
// the work-group's power table (stride QMC_BLOCK).  The four reads are
// independent, so their LDS latencies overlap.
template <typename T>
__device__ __forceinline__ T prod4(uint32_t w, const T *col)
{
    const T a = col[(w & 31u) * QMC_BLOCK];
    const T b = col[((w >> 5) & 31u) * QMC_BLOCK];
    const T c = col[((w >> 10) & 31u) * QMC_BLOCK];
    const T e = col[((w >> 15) & 31u) * QMC_BLOCK];
    return (a * b) * (c * e);
}

// A program word copied into a vector register: the slots are then decoded
// on the vector unit.  The deformed kernel, which reads its derivative
// terms this way, is bound by its scalar unit (shared by the CU's four
// SIMDs) while the vector units idle about half the time.
__device__ __forceinline__ uint32_t to_vgpr(uint32_t w)
{
    uint32_t v;
    asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(w));
    return v;
}

template <typename T>
__device__ __forceinline__ T tmono_lds(cptr<uint32_t> w, const T *col)
{
    const uint32_t w0 = w[0];
    T v = prod4<T>(to_vgpr(w0), col);
    if (w0 >> 30 & 1u) v *= prod4<T>(to_vgpr(w[1]), col);
    return v;
}

} // namespace qmc
