// Device-side building blocks for the FINOM sweeps on gfx950.
//
// Extended-exponent numbers: value = m * 2^e with an FP32 (or FP64) mantissa
// m in [0.5, 1) and an int32 exponent e. They carry the kernel-vector products
// K psi, whose magnitude spans far more than the FP32/FP64 exponent range once
// the potentials are absorbed (section 2.3, remark on log-domain
// stabilisation), while keeping the mantissa's full relative precision.
// Zero is m = 0 with a very negative exponent so that max() in an addition
// always picks the other operand.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace finom {

constexpr int kZeroExp = -(1 << 29);
constexpr int kWave = 64;

template <typename M>
struct Ext {
    M m;
    int e;
};

template <typename M>
__device__ __forceinline__ Ext<M> ext_zero() { return Ext<M>{M(0), kZeroExp}; }

__device__ __forceinline__ float ldexp_m(float m, int e) { return __builtin_amdgcn_ldexpf(m, e); }
__device__ __forceinline__ double ldexp_m(double m, int e) { return __builtin_amdgcn_ldexp(m, e); }
__device__ __forceinline__ float frexp_mant(float m) { return __builtin_amdgcn_frexp_mantf(m); }
__device__ __forceinline__ double frexp_mant(double m) { return __builtin_amdgcn_frexp_mant(m); }
__device__ __forceinline__ int frexp_exp(float m) { return __builtin_amdgcn_frexp_expf(m); }
__device__ __forceinline__ int frexp_exp(double m) { return __builtin_amdgcn_frexp_exp(m); }

// a + b. Both mantissas are scaled to the larger exponent, then renormalised.
template <typename M>
__device__ __forceinline__ Ext<M> ext_add(Ext<M> a, Ext<M> b)
{
    const int e = max(a.e, b.e);
    const M s = ldexp_m(a.m, a.e - e) + ldexp_m(b.m, b.e - e);
    Ext<M> r;
    r.m = frexp_mant(s);
    r.e = (s == M(0)) ? kZeroExp : e + frexp_exp(s);
    return r;
}

template <typename M>
__device__ __forceinline__ Ext<M> ext_mul(Ext<M> a, Ext<M> b)
{
    const M p = a.m * b.m;
    Ext<M> r;
    r.m = frexp_mant(p);
    r.e = (p == M(0)) ? kZeroExp : a.e + b.e + frexp_exp(p);
    return r;
}

// 2^s for an FP64 exponent s (log2 units). s = k + f with k = floor(s),
// f in [0,1); the mantissa is 2^f / 2 in [0.5, 1). Exponents below -2^28
// (including -inf) give zero.
__device__ __forceinline__ float exp2_unit(float f) { return __builtin_amdgcn_exp2f(f); }
__device__ __forceinline__ double exp2_unit(double f) { return exp2(f); }

template <typename M>
__device__ __forceinline__ Ext<M> ext_exp2(double s)
{
    if (!(s > -268435456.0)) return ext_zero<M>();
    s = fmin(s, 268435456.0);
    const double k = floor(s);
    const M m = exp2_unit(static_cast<M>(s - k)) * M(0.5);
    return Ext<M>{m, static_cast<int>(k) + 1};
}

// log2 of an extended value, returned in FP64 (-inf for zero).
__device__ __forceinline__ double log2_unit(float m) { return (double)__builtin_amdgcn_logf(m); }
__device__ __forceinline__ double log2_unit(double m) { return log2(m); }

template <typename M>
__device__ __forceinline__ double ext_log2(Ext<M> a)
{
    if (a.m == M(0)) return -__builtin_inf();
    return log2_unit(a.m) + (double)a.e;
}

// ---------------------------------------------------------------- shuffles

__device__ __forceinline__ float shfl_up_m(float v, int d) { return __shfl_up(v, d, kWave); }
__device__ __forceinline__ double shfl_up_m(double v, int d) { return __shfl_up(v, d, kWave); }
__device__ __forceinline__ float shfl_dn_m(float v, int d) { return __shfl_down(v, d, kWave); }
__device__ __forceinline__ double shfl_dn_m(double v, int d) { return __shfl_down(v, d, kWave); }

template <typename M>
__device__ __forceinline__ Ext<M> shfl_up_ext(Ext<M> v, int d)
{
    return Ext<M>{shfl_up_m(v.m, d), __shfl_up(v.e, d, kWave)};
}

template <typename M>
__device__ __forceinline__ Ext<M> shfl_dn_ext(Ext<M> v, int d)
{
    return Ext<M>{shfl_dn_m(v.m, d), __shfl_down(v.e, d, kWave)};
}

// Exclusive prefix sum (over thread order) and exclusive suffix sum of
// extended values across the block. s_tmp holds 2 * (BLOCK / 64) entries.
// Returns the block totals through the reference arguments.
template <typename M, int BLOCK>
__device__ __forceinline__ void block_scan_both(Ext<M> vl, Ext<M> vu, Ext<M>& excl_l,
                                                Ext<M>& excl_u, Ext<M>& tot_l,
                                                Ext<M>& tot_u, Ext<M>* s_tmp)
{
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    Ext<M> il = vl, iu = vu;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        Ext<M> ol = shfl_up_ext(il, d);
        Ext<M> ou = shfl_dn_ext(iu, d);
        if (lane >= d) il = ext_add(ol, il);
        if (lane + d < kWave) iu = ext_add(iu, ou);
    }
    if (lane == kWave - 1) s_tmp[wid] = il;
    if (lane == 0) s_tmp[NW + wid] = iu;
    __syncthreads();
    Ext<M> pre = ext_zero<M>(), suf = ext_zero<M>();
    Ext<M> tl = ext_zero<M>(), tu = ext_zero<M>();
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        if (w < wid) pre = ext_add(pre, s_tmp[w]);
        if (w > wid) suf = ext_add(suf, s_tmp[NW + w]);
        tl = ext_add(tl, s_tmp[w]);
        tu = ext_add(tu, s_tmp[NW + w]);
    }
    Ext<M> el = shfl_up_ext(il, 1);
    Ext<M> eu = shfl_dn_ext(iu, 1);
    if (lane == 0) el = ext_zero<M>();
    if (lane == kWave - 1) eu = ext_zero<M>();
    excl_l = ext_add(pre, el);
    excl_u = ext_add(eu, suf);
    tot_l = tl;
    tot_u = tu;
}

template <int BLOCK>
__device__ __forceinline__ double block_sum_f64(double v, double* s_tmp)
{
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_down(v, d, kWave);
    if (lane == 0) s_tmp[wid] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += s_tmp[w];
    __syncthreads();
    return t;
}

}  // namespace finom
