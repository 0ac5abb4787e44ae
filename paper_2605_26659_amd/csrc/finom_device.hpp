// Device-side building blocks for the FINOM sweeps on gfx950.
//
// Extended-exponent numbers: value = m * 2^e with an FP32 (or FP64) mantissa
// m and an int32 exponent e. They carry the kernel-vector products K psi,
// whose magnitude spans far more than the FP32/FP64 exponent range once the
// potentials are absorbed (section 2.3, remark on log-domain stabilisation),
// while keeping the mantissa's full relative precision.
//
// Normalisation is lazy: the mantissa is not forced into [0.5, 1). An
// addition aligns both operands to the larger exponent (the smaller operand
// only loses bits it could not contribute anyway), a product multiplies
// mantissas and adds exponents. For the sums of positive terms formed here a
// mantissa grows by at most log2(number of terms), far inside the FP32
// range. Zero is m = 0 with a very negative exponent so that max() in an
// addition always picks the other operand.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace finom {

constexpr int kZeroExp = -(1 << 30);
constexpr double kExpClamp = 134217728.0;   // 2^27: |exponent| bound of ext_exp2
constexpr int kWave = 64;

template <typename M>
struct Ext {
    M m;
    int e;
};

template <typename M>
__device__ __forceinline__ Ext<M> ext_zero() { return Ext<M>{M(0), kZeroExp}; }

// Pointers held in descriptors are generic (flat) pointers to the compiler,
// which then emits flat loads and stores: those also count against the LDS
// wait counter and may alias LDS, so every LDS access after a flat store waits
// for that store to reach memory. All data the kernels touch through
// descriptors lives in device global memory; marking those pointers global
// gives global loads and stores, which the LDS traffic never waits on.
// (The host pass of the compiler parses device functions as well; there the
// qualifier has no meaning and the alias is a plain pointer.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
#else
template <typename T>
using gptr = T*;
#endif

template <typename T>
__device__ __forceinline__ gptr<T> gbl(T* p) { return (gptr<T>)p; }

// A sweep's updated state (always a contiguous run of each line's rows), read
// by the next kernel only, on any XCD: stored non-temporally, so that its lines
// need no write-back from L2 at the kernel's end.
__device__ __forceinline__ void store_update(gptr<double> p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_update(gptr<Ext<float>> p, Ext<float> v)
{
    typedef float f2 __attribute__((ext_vector_type(2)));
    f2 w;
    w.x = v.m;
    w.y = __int_as_float(v.e);
    __builtin_nontemporal_store(w, (gptr<f2>)p);
}

// Workgroups go to the chip's 8 XCDs in turn (workgroup b to XCD b mod 8), and
// each XCD has an L2 of its own. xcd_block renumbers a grid of G workgroups so
// that every XCD takes one contiguous range of work items: neighbouring lines
// of a sweep then meet in one L2 (the strided stores of a 2D sweep fill the
// same cache lines there instead of reaching memory as partial lines).
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_block(int b, int G)
{
    const int q = G / kXcds, r = G % kXcds;
    const int x = b % kXcds, i = b / kXcds;
    return x * q + min(x, r) + i;
}

__device__ __forceinline__ float ldexp_m(float m, int e) { return __builtin_amdgcn_ldexpf(m, e); }
__device__ __forceinline__ double ldexp_m(double m, int e) { return __builtin_amdgcn_ldexp(m, e); }

template <typename M>
__device__ __forceinline__ Ext<M> ext_add(Ext<M> a, Ext<M> b)
{
    const int e = max(a.e, b.e);
    return Ext<M>{ldexp_m(a.m, a.e - e) + ldexp_m(b.m, b.e - e), e};
}

template <typename M>
__device__ __forceinline__ Ext<M> ext_mul(Ext<M> a, Ext<M> b)
{
    return Ext<M>{a.m * b.m, a.e + b.e};
}

// 2^s for an FP64 exponent s (log2 units): s = k + f with k = floor(s),
// f in [0,1), mantissa 2^f in [1, 2). Exponents below -2^27 (including -inf)
// give zero; larger than 2^27 are clamped (no product here gets near either).
__device__ __forceinline__ float exp2_unit(float f) { return __builtin_amdgcn_exp2f(f); }
__device__ __forceinline__ double exp2_unit(double f) { return exp2(f); }

template <typename M>
__device__ __forceinline__ Ext<M> ext_exp2(double s)
{
    if (!(s > -kExpClamp)) return ext_zero<M>();
    s = fmin(s, kExpClamp);
    const double k = floor(s);
    return Ext<M>{exp2_unit(static_cast<M>(s - k)), static_cast<int>(k)};
}

// The same for exponents known to be finite and within +-2^27 (the library
// checks coordinate ranges against eps up front).
template <typename M>
__device__ __forceinline__ Ext<M> ext_exp2_fast(double s)
{
    const double k = floor(s);
    return Ext<M>{exp2_unit(static_cast<M>(s - k)), static_cast<int>(k)};
}

// log2 of an extended value, returned in FP64 (-inf for zero).
__device__ __forceinline__ double log2_unit(float m) { return (double)__builtin_amdgcn_logf(m); }
__device__ __forceinline__ double log2_unit(double m) { return log2(m); }

template <typename M>
__device__ __forceinline__ double ext_log2(Ext<M> a)
{
    if (!(a.m > M(0))) return -__builtin_inf();
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

// ---------------------------------------------------------------- DPP scans
//
// Wavefront-level scans of extended values with data-parallel-primitive moves
// (gfx9 DPP): row_shr/row_shl 1, 2, 4, 8 give scans within each 16-lane row,
// row_bcast:15 and row_bcast:31 carry row totals forward across the 64 lanes;
// the backward direction collects the row totals with readlane. Lanes whose
// DPP source lies outside the row keep the `old` operand, the additive
// identity (mantissa 0, exponent kZeroExp).

template <int CTRL, int RM>
__device__ __forceinline__ int dpp_i(int old, int v)
{
    return __builtin_amdgcn_update_dpp(old, v, CTRL, RM, 0xF, false);
}

template <int CTRL, int RM = 0xF>
__device__ __forceinline__ Ext<float> dpp_ext(Ext<float> v)
{
    return Ext<float>{__int_as_float(dpp_i<CTRL, RM>(0, __float_as_int(v.m))), dpp_i<CTRL, RM>(kZeroExp, v.e)};
}

template <int CTRL, int RM = 0xF>
__device__ __forceinline__ Ext<double> dpp_ext(Ext<double> v)
{
    const long long b = __double_as_longlong(v.m);
    const int lo = dpp_i<CTRL, RM>(0, (int)(b & 0xffffffffLL));
    const int hi = dpp_i<CTRL, RM>(0, (int)(b >> 32));
    return Ext<double>{__longlong_as_double(((long long)hi << 32) | (unsigned int)lo), dpp_i<CTRL, RM>(kZeroExp, v.e)};
}

__device__ __forceinline__ Ext<float> readlane_ext(Ext<float> v, int lane)
{
    return Ext<float>{__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.m), lane)),
                      __builtin_amdgcn_readlane(v.e, lane)};
}

__device__ __forceinline__ Ext<double> readlane_ext(Ext<double> v, int lane)
{
    const long long b = __double_as_longlong(v.m);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return Ext<double>{__longlong_as_double(((long long)hi << 32) | (unsigned int)lo),
                       __builtin_amdgcn_readlane(v.e, lane)};
}

// inclusive prefix sum over the 64 lanes
template <typename M>
__device__ __forceinline__ Ext<M> wave_incl_prefix(Ext<M> v)
{
    v = ext_add(dpp_ext<0x111>(v), v);          // row_shr:1
    v = ext_add(dpp_ext<0x112>(v), v);          // row_shr:2
    v = ext_add(dpp_ext<0x114>(v), v);          // row_shr:4
    v = ext_add(dpp_ext<0x118>(v), v);          // row_shr:8
    v = ext_add(dpp_ext<0x142, 0xA>(v), v);     // row_bcast:15 -> rows 1, 3
    v = ext_add(dpp_ext<0x143, 0xC>(v), v);     // row_bcast:31 -> rows 2, 3
    return v;
}

// inclusive suffix sum over the 64 lanes
template <typename M>
__device__ __forceinline__ Ext<M> wave_incl_suffix(Ext<M> v)
{
    v = ext_add(v, dpp_ext<0x101>(v));          // row_shl:1
    v = ext_add(v, dpp_ext<0x102>(v));          // row_shl:2
    v = ext_add(v, dpp_ext<0x104>(v));          // row_shl:4
    v = ext_add(v, dpp_ext<0x108>(v));          // row_shl:8
    const Ext<M> t1 = readlane_ext(v, 16), t2 = readlane_ext(v, 32), t3 = readlane_ext(v, 48);
    const Ext<M> s2 = t3;
    const Ext<M> s1 = ext_add(t2, t3);
    const Ext<M> s0 = ext_add(t1, s1);
    const int row = (threadIdx.x & (kWave - 1)) >> 4;
    const Ext<M> add = (row == 0) ? s0 : (row == 1) ? s1 : (row == 2) ? s2 : ext_zero<M>();
    return ext_add(v, add);
}

// Exclusive prefix (thread order) and exclusive suffix of extended values over
// the block, with the block totals. s_tmp holds 2 * (BLOCK / 64) entries and
// may be reused once the caller has passed another barrier.
template <typename M, int BLOCK>
__device__ __forceinline__ void block_scan_both(Ext<M> vl, Ext<M> vu, Ext<M>& excl_l,
                                                Ext<M>& excl_u, Ext<M>& tot_l,
                                                Ext<M>& tot_u, Ext<M>* s_tmp)
{
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const Ext<M> il = wave_incl_prefix(vl);
    const Ext<M> iu = wave_incl_suffix(vu);
    if (lane == kWave - 1) s_tmp[wid] = il;
    if (lane == 0) s_tmp[NW + wid] = iu;
    __syncthreads();
    Ext<M> pre = ext_zero<M>(), suf = ext_zero<M>();
    for (int w = 0; w < wid; ++w) pre = ext_add(pre, s_tmp[w]);            // wave-uniform trip count
    for (int w = wid + 1; w < NW; ++w) suf = ext_add(suf, s_tmp[NW + w]);
    Ext<M> el = dpp_ext<0x138>(il);                                         // wave_shr:1
    Ext<M> eu = dpp_ext<0x130>(iu);                                         // wave_shl:1
    excl_l = ext_add(pre, el);
    excl_u = ext_add(eu, suf);
    // totals: prefix of the last lane of the last wave, suffix of lane 0 of wave 0
    tot_l = ext_add(pre, readlane_ext(il, kWave - 1));
    tot_u = ext_add(readlane_ext(iu, 0), suf);
}

// Sum of one extended value per thread; every thread gets the total.
template <typename M, int BLOCK>
__device__ __forceinline__ Ext<M> block_sum_ext(Ext<M> v, Ext<M>* s_tmp)
{
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const Ext<M> w = readlane_ext(wave_incl_prefix(v), kWave - 1);
    __syncthreads();
    if (lane == 0) s_tmp[wid] = w;
    __syncthreads();
    Ext<M> t = ext_zero<M>();
#pragma unroll
    for (int k = 0; k < NW; ++k) t = ext_add(t, s_tmp[k]);
    return t;
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
