// HIP kernels of libsmx for CDNA4 (gfx950, wave64).
//
// The method (paper, Section 2.1): one outer iteration of Algorithm 1 is a
// perturbation phase (trial steps z = x + beta v along v = -grad f/||grad f||,
// beta = gamma alpha^ell, accepted when f does not increase) followed by the
// feasibility step T = box projection of the relaxed simultaneous projection
// onto the bands lower <= Ax <= upper.  T streams A twice: pass 1 reads A row by
// row (r = A z and the band residual t), pass 2 reads the column-major copy
// (A^T of the weighted residual) and applies the box.
//
// Reductions that decide anything (proximity, objective values, gradient norms)
// run in float64 with a fixed order: every workgroup writes its partial sum and
// a one-workgroup kernel launched next sums the partials in workgroup order and
// updates the per-slice state (acceptance of trial steps included).  No kernel
// waits on, or signals, another workgroup of its own grid.
#include <algorithm>
#include <type_traits>
#include "smx_internal.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <math.h>

namespace smx {

// ---------------------------------------------------------------------------
// reductions
//
// A kernel that needs a grid-wide sum writes one partial per workgroup; a
// single-workgroup kernel launched after it sums the partials in workgroup
// order.  Kernel boundaries order the two, so no workgroup ever waits for or
// signals another one, and every sum is reproducible bit for bit.
// ---------------------------------------------------------------------------

// A float64 value moved across lanes by one DPP control (lanes with no source,
// and lanes outside row_mask, receive 0).
template <int CTRL, int ROW_MASK = 0xF>
__device__ inline double dpp_f64(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROW_MASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROW_MASK, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ inline double lane_value(double v, int lane)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes of a wave, returned in every lane.  Register-to-
// register DPP steps: prefix sums inside each row of 16 lanes (shifts by 1, 2,
// 4, 8), then row 0's total into row 1 and row 2's into row 3 (broadcast of
// lane 15), then lane 31's into rows 2 and 3; lane 63 ends with the total.
// The NV sums are independent, so their steps interleave.  Every lane of the
// wave must be active.
template <int NV>
__device__ inline void wave_sum(double (&v)[NV])
{
    constexpr int G = NV < 8 ? NV : 8; // values interleaved at a time (bounds the temporaries)
#pragma unroll
    for (int k0 = 0; k0 < NV; k0 += G) {
#pragma unroll
        for (int k = k0; k < k0 + G && k < NV; ++k) v[k] += dpp_f64<0x111>(v[k]);
#pragma unroll
        for (int k = k0; k < k0 + G && k < NV; ++k) v[k] += dpp_f64<0x112>(v[k]);
#pragma unroll
        for (int k = k0; k < k0 + G && k < NV; ++k) v[k] += dpp_f64<0x114>(v[k]);
#pragma unroll
        for (int k = k0; k < k0 + G && k < NV; ++k) v[k] += dpp_f64<0x118>(v[k]);
#pragma unroll
        for (int k = k0; k < k0 + G && k < NV; ++k) v[k] += dpp_f64<0x142, 0xA>(v[k]);
#pragma unroll
        for (int k = k0; k < k0 + G && k < NV; ++k) v[k] += dpp_f64<0x143, 0xC>(v[k]);
#pragma unroll
        for (int k = k0; k < k0 + G && k < NV; ++k) v[k] = lane_value(v[k], 63);
    }
}

// Sum of v over a workgroup of BS threads, valid in thread 0.  lds holds
// >= (BS/64)*NV doubles.
template <int NV, int BS = kBlock>
__device__ inline void block_sum(double (&v)[NV], double *lds)
{
    wave_sum<NV>(v);
    const int wid = threadIdx.x >> 6, wl = threadIdx.x & 63;
    if (wl == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[wid * NV + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < BS / 64; ++w) s += lds[w * NV + k];
            v[k] = s;
        }
    }
    __syncthreads();
}

// Totals over `count` consecutive slots starting at `first` (each slot NV
// values), summed in slot order by one workgroup of BS threads; valid in
// thread 0.
template <int NV, int BS = kBlock>
__device__ inline void sum_slots(const double *__restrict__ partials, long long first, int count, double (&tot)[NV],
                                 double *lds)
{
#pragma unroll
    for (int k = 0; k < NV; ++k) tot[k] = 0.0;
    for (int b = threadIdx.x; b < count; b += BS) {
#pragma unroll
        for (int k = 0; k < NV; ++k) tot[k] += partials[(first + b) * NV + k];
    }
    block_sum<NV, BS>(tot, lds);
}

// ---------------------------------------------------------------------------
// value loads
// ---------------------------------------------------------------------------

template <typename VT, int VEC>
struct ValLoad;

template <>
struct ValLoad<float, 4> {
    static __device__ inline void load(const void *base, int p, float (&v)[4])
    {
        const float4 q = *reinterpret_cast<const float4 *>(static_cast<const float *>(base) + p);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    }
};

template <>
struct ValLoad<float, 8> {
    static __device__ inline void load(const void *base, int p, float (&v)[8])
    {
        const float4 *q = reinterpret_cast<const float4 *>(static_cast<const float *>(base) + p);
        const float4 a = q[0], b = q[1];
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    }
};

struct Bf16Tag {};
struct F16Tag {};

__device__ inline float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ inline float f16_lo(uint32_t w) { return __half2float(__ushort_as_half((unsigned short)(w & 0xffffu))); }
__device__ inline float f16_hi(uint32_t w) { return __half2float(__ushort_as_half((unsigned short)(w >> 16))); }

template <int VEC>
struct ValLoad16Base {
    static_assert(VEC == 4 || VEC == 8, "VEC");
};

template <>
struct ValLoad<Bf16Tag, 8> {
    static __device__ inline void load(const void *base, int p, float (&v)[8])
    {
        const uint4 q = *reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(base) + p);
        v[0] = bf16_lo(q.x); v[1] = bf16_hi(q.x); v[2] = bf16_lo(q.y); v[3] = bf16_hi(q.y);
        v[4] = bf16_lo(q.z); v[5] = bf16_hi(q.z); v[6] = bf16_lo(q.w); v[7] = bf16_hi(q.w);
    }
};

template <>
struct ValLoad<Bf16Tag, 4> {
    static __device__ inline void load(const void *base, int p, float (&v)[4])
    {
        const uint2 q = *reinterpret_cast<const uint2 *>(static_cast<const uint16_t *>(base) + p);
        v[0] = bf16_lo(q.x); v[1] = bf16_hi(q.x); v[2] = bf16_lo(q.y); v[3] = bf16_hi(q.y);
    }
};

template <>
struct ValLoad<F16Tag, 8> {
    static __device__ inline void load(const void *base, int p, float (&v)[8])
    {
        const uint4 q = *reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(base) + p);
        v[0] = f16_lo(q.x); v[1] = f16_hi(q.x); v[2] = f16_lo(q.y); v[3] = f16_hi(q.y);
        v[4] = f16_lo(q.z); v[5] = f16_hi(q.z); v[6] = f16_lo(q.w); v[7] = f16_hi(q.w);
    }
};

template <>
struct ValLoad<F16Tag, 4> {
    static __device__ inline void load(const void *base, int p, float (&v)[4])
    {
        const uint2 q = *reinterpret_cast<const uint2 *>(static_cast<const uint16_t *>(base) + p);
        v[0] = f16_lo(q.x); v[1] = f16_hi(q.x); v[2] = f16_lo(q.y); v[3] = f16_hi(q.y);
    }
};

template <int VEC>
__device__ inline void idx_load(const int32_t *base, int p, int (&c)[VEC])
{
    const int4 *q = reinterpret_cast<const int4 *>(base + p);
#pragma unroll
    for (int h = 0; h < VEC / 4; ++h) {
        const int4 a = q[h];
        c[4 * h + 0] = a.x; c[4 * h + 1] = a.y; c[4 * h + 2] = a.z; c[4 * h + 3] = a.w;
    }
}

struct Bf16PTag {};
struct F16PTag {};
struct F32U16Tag {}; // float32 values beside a uint16 index array

// VEC entries (values as float, indices) starting at p.
template <typename VT, int VEC>
struct Entries {
    static __device__ inline void load(const SpView &A, int p, float (&v)[VEC], int (&c)[VEC])
    {
        ValLoad<VT, VEC>::load(A.val, p, v);
        idx_load<VEC>(A.idx, p, c);
    }
};

template <int VEC, bool BF>
__device__ inline void packed_load(const SpView &A, int p, float (&v)[VEC], int (&c)[VEC])
{
    const uint4 *q = reinterpret_cast<const uint4 *>(static_cast<const uint32_t *>(A.val) + p);
#pragma unroll
    for (int h = 0; h < VEC / 4; ++h) {
        const uint4 a = q[h];
        const uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[4 * h + k] = BF ? bf16_lo(w[k]) : f16_lo(w[k]);
            c[4 * h + k] = (int)(w[k] >> 16);
        }
    }
}

template <int VEC>
struct Entries<F32U16Tag, VEC> {
    static __device__ inline void load(const SpView &A, int p, float (&v)[VEC], int (&c)[VEC])
    {
        ValLoad<float, VEC>::load(A.val, p, v);
        const uint16_t *ib = reinterpret_cast<const uint16_t *>(A.idx) + p;
        if constexpr (VEC == 4) {
            const uint2 a = *reinterpret_cast<const uint2 *>(ib);
            c[0] = (int)(a.x & 0xFFFFu); c[1] = (int)(a.x >> 16); c[2] = (int)(a.y & 0xFFFFu); c[3] = (int)(a.y >> 16);
        } else {
            const uint4 a = *reinterpret_cast<const uint4 *>(ib);
            const uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                c[2 * k] = (int)(w[k] & 0xFFFFu);
                c[2 * k + 1] = (int)(w[k] >> 16);
            }
        }
    }
};

template <int VEC>
struct Entries<Bf16PTag, VEC> {
    static __device__ inline void load(const SpView &A, int p, float (&v)[VEC], int (&c)[VEC])
    {
        packed_load<VEC, true>(A, p, v, c);
    }
};

template <int VEC>
struct Entries<F16PTag, VEC> {
    static __device__ inline void load(const SpView &A, int p, float (&v)[VEC], int (&c)[VEC])
    {
        packed_load<VEC, false>(A, p, v, c);
    }
};

// VEC stored entries at p as loaded, before any arithmetic on them (the
// bit patterns of the values, the index words), and their decoding.  Loops
// that keep several chunks in flight issue every chunk's loads first, each
// under its own predicate, and decode afterwards: a decode inside the
// predicated block would wait for that chunk's load before the next chunk's
// loads are issued, one memory round trip per chunk.  A chunk left
// unloaded decodes to value 0 at index 0.
template <typename VT, int VEC>
struct EntryRaw {
    static_assert(VEC == 4 || VEC == 8, "VEC");
    static constexpr int NV = std::is_same<VT, float>::value || std::is_same<VT, F32U16Tag>::value ? VEC
                              : (std::is_same<VT, Bf16PTag>::value || std::is_same<VT, F16PTag>::value) ? VEC
                                                                                                          : VEC / 2;
    static constexpr bool kIdx32 = !(std::is_same<VT, F32U16Tag>::value || std::is_same<VT, Bf16PTag>::value ||
                                     std::is_same<VT, F16PTag>::value);
    static constexpr int NI = kIdx32 ? VEC : (std::is_same<VT, F32U16Tag>::value ? VEC / 2 : 0);
    uint32_t vw[NV];
    uint32_t iw[NI > 0 ? NI : 1];

    __device__ inline void zero()
    {
#pragma unroll
        for (int k = 0; k < NV; ++k) vw[k] = 0u;
#pragma unroll
        for (int k = 0; k < (NI > 0 ? NI : 1); ++k) iw[k] = 0u;
    }
    __device__ inline void load(const SpView &A, int p)
    {
        if constexpr (std::is_same<VT, Bf16PTag>::value || std::is_same<VT, F16PTag>::value) {
            const uint4 *q = reinterpret_cast<const uint4 *>(static_cast<const uint32_t *>(A.val) + p);
#pragma unroll
            for (int h = 0; h < VEC / 4; ++h) {
                const uint4 a = q[h];
                vw[4 * h] = a.x; vw[4 * h + 1] = a.y; vw[4 * h + 2] = a.z; vw[4 * h + 3] = a.w;
            }
        } else {
            if constexpr (NV == VEC) { // 32-bit values
                const uint4 *q = reinterpret_cast<const uint4 *>(static_cast<const uint32_t *>(A.val) + p);
#pragma unroll
                for (int h = 0; h < VEC / 4; ++h) {
                    const uint4 a = q[h];
                    vw[4 * h] = a.x; vw[4 * h + 1] = a.y; vw[4 * h + 2] = a.z; vw[4 * h + 3] = a.w;
                }
            } else { // 16-bit values, two a word
                const uint16_t *b = static_cast<const uint16_t *>(A.val) + p;
                if constexpr (VEC == 8) {
                    const uint4 a = *reinterpret_cast<const uint4 *>(b);
                    vw[0] = a.x; vw[1] = a.y; vw[2] = a.z; vw[3] = a.w;
                } else {
                    const uint2 a = *reinterpret_cast<const uint2 *>(b);
                    vw[0] = a.x; vw[1] = a.y;
                }
            }
            if constexpr (kIdx32) {
                const uint4 *q = reinterpret_cast<const uint4 *>(A.idx + p);
#pragma unroll
                for (int h = 0; h < VEC / 4; ++h) {
                    const uint4 a = q[h];
                    iw[4 * h] = a.x; iw[4 * h + 1] = a.y; iw[4 * h + 2] = a.z; iw[4 * h + 3] = a.w;
                }
            } else { // 16-bit indices, two a word
                const uint16_t *ib = reinterpret_cast<const uint16_t *>(A.idx) + p;
                if constexpr (VEC == 8) {
                    const uint4 a = *reinterpret_cast<const uint4 *>(ib);
                    iw[0] = a.x; iw[1] = a.y; iw[2] = a.z; iw[3] = a.w;
                } else {
                    const uint2 a = *reinterpret_cast<const uint2 *>(ib);
                    iw[0] = a.x; iw[1] = a.y;
                }
            }
        }
    }
    __device__ inline void decode(float (&v)[VEC], int (&c)[VEC]) const
    {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            if constexpr (std::is_same<VT, Bf16PTag>::value) {
                v[e] = bf16_lo(vw[e]);
                c[e] = (int)(vw[e] >> 16);
            } else if constexpr (std::is_same<VT, F16PTag>::value) {
                v[e] = f16_lo(vw[e]);
                c[e] = (int)(vw[e] >> 16);
            } else {
                if constexpr (NV == VEC) v[e] = __uint_as_float(vw[e]);
                else if constexpr (std::is_same<VT, Bf16Tag>::value) v[e] = (e & 1) ? bf16_hi(vw[e >> 1]) : bf16_lo(vw[e >> 1]);
                else v[e] = (e & 1) ? f16_hi(vw[e >> 1]) : f16_lo(vw[e >> 1]);
                if constexpr (kIdx32) c[e] = (int)iw[e];
                else c[e] = (int)((e & 1) ? (iw[e >> 1] >> 16) : (iw[e >> 1] & 0xFFFFu));
            }
        }
    }
};

// U chunks of VEC entries (chunk u at p + u * step, loaded where ok[u]):
// every load issued, then every chunk decoded.
template <typename VT, int VEC, int U>
__device__ inline void load_chunks(const SpView &A, int p, int step, const bool (&ok)[U], float (&v)[U][VEC],
                                   int (&c)[U][VEC])
{
    EntryRaw<VT, VEC> raw[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        raw[u].zero();
        if (ok[u]) raw[u].load(A, p + u * step);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) raw[u].decode(v[u], c[u]);
}

// One entry at p: its value as float and its index.
template <typename VT>
__device__ inline void entry1(const SpView &A, int p, float &v, int &c);
template <>
__device__ inline void entry1<float>(const SpView &A, int p, float &v, int &c)
{
    v = static_cast<const float *>(A.val)[p];
    c = A.idx[p];
}
template <>
__device__ inline void entry1<Bf16Tag>(const SpView &A, int p, float &v, int &c)
{
    v = bf16_lo(static_cast<const uint16_t *>(A.val)[p]);
    c = A.idx[p];
}
template <>
__device__ inline void entry1<F16Tag>(const SpView &A, int p, float &v, int &c)
{
    v = f16_lo(static_cast<const uint16_t *>(A.val)[p]);
    c = A.idx[p];
}
template <>
__device__ inline void entry1<Bf16PTag>(const SpView &A, int p, float &v, int &c)
{
    const uint32_t w = static_cast<const uint32_t *>(A.val)[p];
    v = bf16_lo(w);
    c = (int)(w >> 16);
}
template <>
__device__ inline void entry1<F16PTag>(const SpView &A, int p, float &v, int &c)
{
    const uint32_t w = static_cast<const uint32_t *>(A.val)[p];
    v = f16_lo(w);
    c = (int)(w >> 16);
}
template <>
__device__ inline void entry1<F32U16Tag>(const SpView &A, int p, float &v, int &c)
{
    v = static_cast<const float *>(A.val)[p];
    c = reinterpret_cast<const uint16_t *>(A.idx)[p];
}

// Partial dot product of one row with a vector, lanes interleaved: lane l of
// an LPR-lane group takes entries beg + l, beg + l + LPR, ...  Neighbouring
// lanes read neighbouring entries (one coalesced load per instruction), and
// their gathers land on neighbouring entries of the row, which for a ray are
// often neighbouring pixels in one cache line.  Eight entries per lane in
// flight; entries past the row's end are skipped (LPR may exceed the row
// alignment).
template <int LPR, typename VT>
__device__ inline double row_dot_interleaved(const SpView &A, int beg, int end, int lane, const float *__restrict__ x)
{
    constexpr int U = 8;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int p = beg + lane;
    for (; p + (U - 1) * LPR < end; p += U * LPR) {
        float v[U];
        int c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) entry1<VT>(A, p + u * LPR, v[u], c[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u & 3] = fma((double)v[u], (double)x[c[u]], acc[u & 3]);
    }
    for (; p < end; p += LPR) {
        float v0;
        int c0;
        entry1<VT>(A, p, v0, c0);
        acc[0] = fma((double)v0, (double)x[c0], acc[0]);
    }
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// Partial dot product of one row with a vector, by lane `lane` of an LPR-lane
// group.  [beg, end) is row-aligned, so every vector load is aligned and no
// entry needs a mask (padding entries are zeros with valid indices).  Products
// of two float32 numbers are exact in float64, so accumulating in float64
// leaves only the rounding of the sums; the pass is bound by memory traffic,
// not by the float64 rate.
template <int LPR, int VEC, typename VT>
__device__ inline double row_dot_chunked(const SpView &A, int beg, int end, int lane, const float *__restrict__ x)
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int p = beg + lane * VEC;
    constexpr int STEP = LPR * VEC;
    // four independent loads in flight per lane; the row's last chunks (fewer
    // than four) are issued together as well, each under its own predicate,
    // so a row costs one load-then-gather round trip per four chunks
    for (; p < end; p += 4 * STEP) {
        float v[4][VEC];
        int c[4][VEC];
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) ok[u] = p + u * STEP < end;
        load_chunks<VT, VEC, 4>(A, p, STEP, ok, v, c);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (ok[u]) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc[u] = fma((double)v[u][e], (double)x[c[u][e]], acc[u]);
            }
    }
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// VEC 1: interleaved lanes; otherwise chunks of VEC entries per lane.
template <int LPR, int VEC, typename VT>
__device__ inline double row_dot(const SpView &A, int beg, int end, int lane, const float *__restrict__ x)
{
    if constexpr (VEC == 1) return row_dot_interleaved<LPR, VT>(A, beg, end, lane, x);
    else return row_dot_chunked<LPR, VEC, VT>(A, beg, end, lane, x);
}

template <int LPR>
__device__ inline double group_sum(double v)
{
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, LPR);
    return v;
}

// ---------------------------------------------------------------------------
// pass 1: r = A z, t = clip(r, lower, upper) - r, c = S t, and one partial of
// the proximity 1/2 sum D t^2 per workgroup (or, in quadratic-form mode, of
// sum S r^2)
// ---------------------------------------------------------------------------

// Pass-1 epilogue of row `row` (slice s of B) from r = <a_i, v>: returns the
// row's partial term and stores c_i (not in quadratic-form mode).  With S = D
// this is exactly c_i = D_i t_i and the term D_i t_i^2.  A dose-volume row
// only keeps r: its bands are set after the pass, and the dose-volume kernels
// write its c_i and its proximity term.
__device__ inline double epi1(const RowW &w, double r, float lo, float up, float d, float sw, float *c,
                              long long row, int s, int B)
{
    if (w.qform) return (double)sw * r * r;
    if (w.dose && row >= w.dose_lo && row < w.dose_hi) {
        w.dose[(row - w.dose_lo) * B + s] = r;
        return 0.0;
    }
    const double t = fmin(fmax(r, (double)lo), (double)up) - r;
    const double dt = (double)d * t;
    *c = (float)((double)sw * t);
    return dt * t;
}

template <int LPR, int VEC, typename VT>
__global__ __launch_bounds__(kBlock) void k_pass1(SpView A, const float *__restrict__ x,
                                                  const float *__restrict__ lower, const float *__restrict__ upper,
                                                  RowW w, float *__restrict__ c,
                                                  const SliceState *__restrict__ st, int query,
                                                  double *__restrict__ partials)
{
    __shared__ double lds[4];
    constexpr int RPB = kBlock / LPR;
    const int lane = threadIdx.x & (LPR - 1);
    const int grp = threadIdx.x / LPR;
    const bool live = query ? true : st[0].live != 0;
    double pacc[1] = {0.0};
    if (live) {
        const long long stride = (long long)gridDim.x * RPB;
        long long row = (long long)blockIdx.x * RPB + grp;
        int beg = 0, end = 0;
        if (row < A.rows) {
            beg = A.ptr[row];
            end = A.ptr[row + 1];
        }
        for (; row < A.rows; row += stride) {
            int nbeg = 0, nend = 0; // the next row's offsets, in flight meanwhile
            if (row + stride < A.rows) {
                nbeg = A.ptr[row + stride];
                nend = A.ptr[row + stride + 1];
            }
            // epilogue operands, fetched while the row streams (every lane of the
            // group reads the same words: no predicated block whose conversions
            // would wait for them before the row's loads are issued)
            const float lo = lower[row], up = upper[row], d = w.D[row], sw = w.S[row];
            const double r = group_sum<LPR>(row_dot<LPR, VEC, VT>(A, beg, end, lane, x)) * (double)A.vscale_inv;
            if (lane == 0) pacc[0] += epi1(w, r, lo, up, d, sw, c + row, row, 0, 1);
            beg = nbeg;
            end = nend;
        }
    }
    block_sum<1>(pacc, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = pacc[0];
}

// Copies v[0, P) into LDS (dst, 16-byte aligned) with BS threads: float4
// loads, four in flight per thread (every load in bounds: past the end the
// last float4 is read again, and not stored), then the last P mod 4 values.
template <int BS>
__device__ inline void stage_vector(float4 *dst, const float *__restrict__ v, int P)
{
    const int q4 = P >> 2;
    const float4 *v4 = reinterpret_cast<const float4 *>(v);
    for (int e0 = threadIdx.x; e0 < q4; e0 += 4 * BS) {
        float4 t[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) t[u] = v4[min(e0 + u * BS, q4 - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (e0 + u * BS < q4) dst[e0 + u * BS] = t[u];
    }
    if (threadIdx.x < (P & 3)) reinterpret_cast<float *>(dst)[4 * q4 + threadIdx.x] = v[4 * q4 + threadIdx.x];
}

// One unknown of the linear objective's trial point z = x + s v, v = -c/||c||
// (inv_gn = 1/||c||): the one expression every kernel forming z uses, so the
// pass that stages z and the apply kernel that forms it again agree bit for bit.
__device__ inline float linear_step_point(float xj, float cj, double s_acc, double inv_gn)
{
    return (float)((double)xj + s_acc * (-(double)cj * inv_gn));
}

// stage_vector of z = x + s v for the linear objective (x and c both read as
// float4, four loads of each in flight per thread).
template <int BS>
__device__ inline void stage_linear_point(float4 *dst, const float *__restrict__ x, const float *__restrict__ c, int P,
                                          double s_acc, double inv_gn)
{
    const int q4 = P >> 2;
    const float4 *x4 = reinterpret_cast<const float4 *>(x);
    const float4 *c4 = reinterpret_cast<const float4 *>(c);
    for (int e0 = threadIdx.x; e0 < q4; e0 += 4 * BS) {
        float4 tx[4], tc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            tx[u] = x4[min(e0 + u * BS, q4 - 1)];
            tc[u] = c4[min(e0 + u * BS, q4 - 1)];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (e0 + u * BS < q4)
                dst[e0 + u * BS] = make_float4(linear_step_point(tx[u].x, tc[u].x, s_acc, inv_gn),
                                               linear_step_point(tx[u].y, tc[u].y, s_acc, inv_gn),
                                               linear_step_point(tx[u].z, tc[u].z, s_acc, inv_gn),
                                               linear_step_point(tx[u].w, tc[u].w, s_acc, inv_gn));
    }
    if (threadIdx.x < (P & 3)) {
        const int j = 4 * q4 + threadIdx.x;
        reinterpret_cast<float *>(dst)[j] = linear_step_point(x[j], c[j], s_acc, inv_gn);
    }
}

// Row dot product whose gathers read the vector's first P entries from an
// LDS copy (xl) and the rest from memory; otherwise row_dot_chunked.
template <int LPR, int VEC, typename VT>
__device__ inline double row_dot_split(const SpView &A, int beg, int end, int lane, const float *__restrict__ x,
                                       const float *xl, int P)
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int p = beg + lane * VEC;
    constexpr int STEP = LPR * VEC;
    for (; p < end; p += 4 * STEP) {
        float v[4][VEC];
        int c[4][VEC];
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) ok[u] = p + u * STEP < end;
        load_chunks<VT, VEC, 4>(A, p, STEP, ok, v, c);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (ok[u]) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const int ci = c[u][e];
                    float xv;
                    if (ci < P) xv = xl[ci];
                    else xv = x[ci];
                    acc[u] = fma((double)v[u][e], (double)xv, acc[u]);
                }
            }
    }
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// Pass 1 with the gathered vector partly in LDS.  A gather through the
// vector memory path costs about one address per CU per clock, whatever its
// locality; an LDS read serves many lanes per clock.  So each workgroup (one
// per CU, 1024 threads) first copies x[0, P) into LDS, P = min(n, 40,448),
// then runs the rows as k_pass1 does, gathering x_j from LDS when j < P.
template <int LPR, int VEC, typename VT>
__global__ __launch_bounds__(kLdsPassBlock) void k_pass1_lds(SpView A, const float *__restrict__ x, int P,
                                                              const float *__restrict__ lower,
                                                              const float *__restrict__ upper, RowW w,
                                                              float *__restrict__ c,
                                                              const SliceState *__restrict__ st, int query,
                                                              double *__restrict__ partials)
{
    extern __shared__ float4 xl4[];
    float *xl = reinterpret_cast<float *>(xl4);
    __shared__ double lds[kLdsPassBlock / 64];
    constexpr int RPB = kLdsPassBlock / LPR;
    const int lane = threadIdx.x & (LPR - 1);
    const int grp = threadIdx.x / LPR;
    const bool live = query ? true : st[0].live != 0; // the same in every thread
    double pacc[1] = {0.0};
    if (live) {
        stage_vector<kLdsPassBlock>(xl4, x, P);
        __syncthreads();
        const long long stride = (long long)gridDim.x * RPB;
        long long row = (long long)blockIdx.x * RPB + grp;
        int beg = 0, end = 0;
        if (row < A.rows) {
            beg = A.ptr[row];
            end = A.ptr[row + 1];
        }
        for (; row < A.rows; row += stride) {
            int nbeg = 0, nend = 0; // the next row's offsets, in flight meanwhile
            if (row + stride < A.rows) {
                nbeg = A.ptr[row + stride];
                nend = A.ptr[row + stride + 1];
            }
            const float lo = lower[row], up = upper[row], d = w.D[row], sw = w.S[row]; // read by every lane
            const double r =
                group_sum<LPR>(row_dot_split<LPR, VEC, VT>(A, beg, end, lane, x, xl, P)) * (double)A.vscale_inv;
            if (lane == 0) pacc[0] += epi1(w, r, lo, up, d, sw, c + row, row, 0, 1);
            beg = nbeg;
            end = nend;
        }
    }
    block_sum<1, kLdsPassBlock>(pacc, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = pacc[0];
}

// ---------------------------------------------------------------------------
// Streaming pass kernels.  A workgroup takes one row block (at most
// kStreamEntries entries): every lane issues all of its value/index loads and
// gathers at once, the exact float64 products go to LDS, and each row is then
// summed from LDS by a group of G lanes (G the largest power of two with
// G * rows <= kBlock).  A row longer than a block is summed by the whole
// workgroup.  Rows of one block are consecutive, so the loads are one
// contiguous stream per workgroup.
// ---------------------------------------------------------------------------

struct RowSplit {
    int G, rl, lane;
};

__device__ inline RowSplit split_rows(int nr)
{
    int G = 64;
    while (G > 1 && G * nr > kBlock) G >>= 1;
    RowSplit r;
    r.G = G;
    r.rl = threadIdx.x / G;
    r.lane = threadIdx.x & (G - 1);
    return r;
}

// Sums of the VEC-entry chunks of [e0, e1) with v: chunk j (entries e0 + j*VEC
// ..) into prod[j].  Rows start at multiples of kRowAlign (a multiple of VEC),
// so no chunk straddles two rows; each product of two float32 numbers is exact
// in float64.
template <int VEC, typename VT>
__device__ inline void stream_chunks(const SpView &A, int e0, int e1, const float *__restrict__ v, double *prod)
{
    constexpr int PER = kStreamEntries / (kBlock * VEC);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int j = k * kBlock + threadIdx.x;
        const int q = j * VEC;
        if (e0 + q < e1) {
            float val[VEC];
            int id[VEC];
            Entries<VT, VEC>::load(A, e0 + q, val, id);
            double acc = 0.0;
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc = fma((double)val[e], (double)v[id[e]], acc);
            prod[j] = acc;
        }
    }
}

// Sum over lanes of the G-lane group (every thread of the workgroup calls it).
__device__ inline double group_sum_rt(double s, int G)
{
    for (int off = G >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off, G);
    return s;
}

// Whole-workgroup sum of one long row; valid in thread 0.
template <int VEC, typename VT>
__device__ inline double long_row_sum(const SpView &A, int e0, int e1, const float *__restrict__ v, double *lds)
{
    double acc = 0.0;
    for (int p = e0 + threadIdx.x * VEC; p < e1; p += kBlock * VEC) {
        float val[VEC];
        int id[VEC];
        Entries<VT, VEC>::load(A, p, val, id);
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc = fma((double)val[e], (double)v[id[e]], acc);
    }
    double t[1] = {acc};
    block_sum<1>(t, lds);
    return t[0];
}

template <int VEC, typename VT>
__global__ __launch_bounds__(kBlock) void k_pass1_stream(SpView A, RowBlocks RB, const float *__restrict__ x,
                                                         const float *__restrict__ lower,
                                                         const float *__restrict__ upper,
                                                         RowW w, float *__restrict__ c,
                                                         const SliceState *__restrict__ st, int query,
                                                         double *__restrict__ partials)
{
    __shared__ double prod[kStreamEntries / VEC];
    __shared__ int rp[kBlock + 1];
    __shared__ double lds[4];
    const bool live = query ? true : st[0].live != 0;
    double pacc[1] = {0.0};
    if (live) {
        for (int b = blockIdx.x; b < RB.nblk; b += gridDim.x) {
            const int r0 = RB.rb[b], r1 = RB.rb[b + 1];
            const int e0 = A.ptr[r0], e1 = A.ptr[r1];
            if (e1 - e0 > kStreamEntries) {
                const double sum = long_row_sum<VEC, VT>(A, e0, e1, x, lds);
                if (threadIdx.x == 0)
                    pacc[0] += epi1(w, sum * (double)A.vscale_inv, lower[r0], upper[r0], w.D[r0], w.S[r0], c + r0,
                                    r0, 0, 1);
                continue;
            }
            const int nr = r1 - r0;
            const RowSplit rs = split_rows(nr);
            const bool owner = rs.rl < nr && rs.lane == 0;
            float lo = 0.f, up = 0.f, d = 0.f, sw = 0.f;
            if (owner) { // epilogue operands, fetched while the products stream
                lo = lower[r0 + rs.rl];
                up = upper[r0 + rs.rl];
                d = w.D[r0 + rs.rl];
                sw = w.S[r0 + rs.rl];
            }
            for (int i = threadIdx.x; i <= nr; i += kBlock) rp[i] = (A.ptr[r0 + i] - e0) / VEC;
            stream_chunks<VEC, VT>(A, e0, e1, x, prod);
            __syncthreads();
            double s = 0.0;
            if (rs.rl < nr)
                for (int q = rp[rs.rl] + rs.lane; q < rp[rs.rl + 1]; q += rs.G) s += prod[q];
            s = group_sum_rt(s, rs.G);
            if (owner) pacc[0] += epi1(w, s * (double)A.vscale_inv, lo, up, d, sw, c + r0 + rs.rl, r0 + rs.rl, 0, 1);
            __syncthreads();
        }
    }
    block_sum<1>(pacc, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = pacc[0];
}

__device__ inline double nan64() { return __longlong_as_double(0x7ff8000000000000LL); }

// ---------------------------------------------------------------------------
// State buffers.  Every kernel reads the per-slice states from st_in; kernels
// that advance the state have exactly one writer per slice (thread 0 of the
// slice's workgroup 0), which writes the whole new state to the other buffer
// st_out.  The host alternates the two buffers launch by launch, so a kernel
// never reads a state another workgroup of the same grid is writing.
// ---------------------------------------------------------------------------

// Whether a slice runs its next iteration.
__device__ inline int slice_runs(const SliceState &S)
{
    return (S.enabled && S.k < S.k_end && S.stop_reason == STOP_NONE) ? 1 : 0;
}

// Stopping rules after a feasibility step that recorded proximity `prox`
// (Section 2.2.1: P <= P*, or |P^{k+1} - P^k| / max{1, P^k} < Delta P* for N
// consecutive iterations, or N_max iterations).  A superiorized run (a phase
// ran, so f_start = f(x^k) is set) only notes whether a proximity rule held;
// its objective condition is checked when the next phase opens.  The variance
// rule follows in k_stop_var.
__device__ inline void stop_rules_after_step(SliceState &S, double prox)
{
    if (!isnan(S.p_last)) {
        const double dp = fabs(prox - S.p_last) / fmax(1.0, S.p_last);
        S.dp_run = dp < S.stop_dprox ? S.dp_run + 1 : 0;
    }
    S.p_last = prox;
    const bool by_prox = prox <= S.stop_prox, by_dprox = S.dp_run >= S.stop_n;
    if (!isnan(S.f_start)) {
        S.feas_ok = (by_prox || by_dprox) ? 1 : 0;
        S.f_last = S.f_start;
    } else if (by_prox) {
        S.stop_reason = STOP_PROX;
    } else if (by_dprox) {
        S.stop_reason = STOP_DPROX;
    }
    if (S.stop_reason == STOP_NONE && S.stop_max > 0 && S.k >= S.stop_max) S.stop_reason = STOP_MAXIT;
}

// End of an outer iteration: proximity from pass 1's partials, the history
// record, k + 1, and whether the next iteration runs.  Called by every thread
// of one workgroup (BS threads; lds holds BS/64 doubles).
template <int BS = kBlock>
__device__ inline void finish_iteration(const SliceState *__restrict__ st_in, SliceState *__restrict__ st_out, int B,
                                        const double *__restrict__ part1, int nparts, const Hist &h, double *lds)
{
    for (int s = 0; s < B; ++s) {
        double tot[1];
        sum_slots<1, BS>(part1, (long long)s * nparts, nparts, tot, lds);
        if (threadIdx.x == 0) {
            SliceState S = st_in[s];
            S.ran = S.live;
            if (S.live) {
                const double prox = 0.5 * tot[0];
                S.prox = prox;
                if (!isfinite(prox)) S.nonfinite = 1;
                if (S.k < h.cap) {
                    const long long r = S.k * B + s;
                    h.prox[r] = prox;
                    h.f_start[r] = S.f_start;
                    h.f_end[r] = S.f_cur;
                    h.trials[r] = S.trials_it;
                    h.accepts[r] = S.accepts_it;
                }
                S.k += 1;
                if (S.stop_on) stop_rules_after_step(S, prox);
            }
            if (!isnan(S.f_cur)) S.f_ref = S.f_cur; // where this iteration's phase ended
            S.f_start = S.f_cur = nan64();
            S.trials_it = 0;
            S.accepts_it = 0;
            S.phase = 0;
            S.live = slice_runs(S);
            st_out[s] = S;
        }
    }
}

// ---------------------------------------------------------------------------
// pass 2: y = A^T c, x = clip(z + lambda y, lo, hi) (DROP: lambda Z_j y);
// workgroup 0 also closes the outer iteration.  For the extrapolated steps
// (deferred mode) y itself is kept, with per-workgroup partials of ||y||^2,
// and k_step_apply updates x and closes the iteration.
// ---------------------------------------------------------------------------

// Pass-2 epilogue of one column (x and ybuf index e); returns y^2 in deferred
// mode, else 0.
__device__ inline double epi2(const ColStep &cs, long long col, long long e, double y, float xo, float l, float u,
                              float *__restrict__ x)
{
    if (cs.defer) {
        cs.ybuf[e] = y;
        if (cs.ybuf32) cs.ybuf32[e] = (float)y;
        return y * y;
    }
    const double yy = cs.zcol ? y * (double)cs.zcol[col] : y;
    const double z = fma((double)cs.lambda, yy, (double)xo);
    x[e] = (float)fmin(fmax(z, (double)l), (double)u);
    return 0.0;
}

// End of a pass-2 launch (workgroups of BS threads): the ||y||^2 partials
// (deferred mode), else workgroup 0 closes the outer iteration.
template <int BS = kBlock>
__device__ inline void end_pass2(const ColStep &cs, double yacc, const SliceState *__restrict__ st_in,
                                 SliceState *__restrict__ st_out, const double *__restrict__ part1, int nparts1,
                                 const Hist &h, double *lds)
{
    if (cs.defer) {
        double v[1] = {yacc};
        block_sum<1, BS>(v, lds);
        if (threadIdx.x == 0) cs.ypart[blockIdx.x] = v[0];
    } else if (blockIdx.x == 0) {
        finish_iteration<BS>(st_in, st_out, 1, part1, nparts1, h, lds);
    }
}

template <int LPR, int VEC, typename VT>
__global__ __launch_bounds__(kBlock) void k_pass2(SpView At, const float *__restrict__ c, float *__restrict__ x,
                                                  ColStep cs, const SliceState *__restrict__ st_in,
                                                  SliceState *__restrict__ st_out, const double *__restrict__ part1,
                                                  int nparts1, Hist h)
{
    __shared__ double lds[4];
    constexpr int RPB = kBlock / LPR;
    double yacc = 0.0;
    if (st_in[0].live) {
        const int lane = threadIdx.x & (LPR - 1);
        const int grp = threadIdx.x / LPR;
        const long long stride = (long long)gridDim.x * RPB;
        for (long long col = (long long)blockIdx.x * RPB + grp; col < At.rows; col += stride) {
            const int beg = At.ptr[col], end = At.ptr[col + 1];
            float xo = 0.f, l = 0.f, u = 0.f;
            if (lane == 0 && !cs.defer) { // epilogue operands, fetched while the column streams
                xo = x[col];
                l = cs.lo[col];
                u = cs.hi[col];
            }
            const double y = group_sum<LPR>(row_dot<LPR, VEC, VT>(At, beg, end, lane, c)) * (double)At.vscale_inv;
            if (lane == 0) yacc += epi2(cs, col, col, y, xo, l, u, x);
        }
    }
    end_pass2(cs, yacc, st_in, st_out, part1, nparts1, h, lds);
}

// Pass 2 with the gathered residual partly in LDS, as k_pass1_lds: one
// workgroup per CU copies c[0, P) into LDS, P = min(m, 40,448), then sums
// each column as k_pass2 does, reading c_i from LDS when i < P.
template <int LPR, int VEC, typename VT>
__global__ __launch_bounds__(kLdsPassBlock) void k_pass2_lds(SpView At, const float *__restrict__ c, int P,
                                                             float *__restrict__ x, ColStep cs,
                                                             const SliceState *__restrict__ st_in,
                                                             SliceState *__restrict__ st_out,
                                                             const double *__restrict__ part1, int nparts1, Hist h)
{
    extern __shared__ float4 cl4[];
    float *cl = reinterpret_cast<float *>(cl4);
    __shared__ double lds[kLdsPassBlock / 64];
    constexpr int RPB = kLdsPassBlock / LPR;
    double yacc = 0.0;
    if (st_in[0].live) { // the same in every thread
        stage_vector<kLdsPassBlock>(cl4, c, P);
        __syncthreads();
        const int lane = threadIdx.x & (LPR - 1);
        const int grp = threadIdx.x / LPR;
        const long long stride = (long long)gridDim.x * RPB;
        long long col = (long long)blockIdx.x * RPB + grp;
        int beg = 0, end = 0;
        if (col < At.rows) {
            beg = At.ptr[col];
            end = At.ptr[col + 1];
        }
        for (; col < At.rows; col += stride) {
            int nbeg = 0, nend = 0; // the next column's offsets, in flight meanwhile
            if (col + stride < At.rows) {
                nbeg = At.ptr[col + stride];
                nend = At.ptr[col + stride + 1];
            }
            float xo = 0.f, l = 0.f, u = 0.f;
            if (lane == 0 && !cs.defer) {
                xo = x[col];
                l = cs.lo[col];
                u = cs.hi[col];
            }
            const double y =
                group_sum<LPR>(row_dot_split<LPR, VEC, VT>(At, beg, end, lane, c, cl, P)) * (double)At.vscale_inv;
            if (lane == 0) yacc += epi2(cs, col, col, y, xo, l, u, x);
            beg = nbeg;
            end = nend;
        }
    }
    end_pass2<kLdsPassBlock>(cs, yacc, st_in, st_out, part1, nparts1, h, lds);
}

// Sum of one column segment [beg, end) of the column copy whose rows all lie
// in the panel staged in LDS (cl[row - base]).  Segments start anywhere in a
// column, so the chunks start at the aligned position before beg and the
// entries outside [beg, end) are masked (they are in bounds: a column is
// padded to a multiple of kRowAlign entries).
template <int LPR, int VEC, typename VT>
__device__ inline double seg_dot_lds(const SpView &A, int beg, int end, int lane, const float *cl, int base)
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    constexpr int STEP = LPR * VEC;
    for (int p = (beg / VEC) * VEC + lane * VEC; p < end; p += 4 * STEP) {
        float v[4][VEC];
        int c[4][VEC];
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) ok[u] = p + u * STEP < end;
        load_chunks<VT, VEC, 4>(A, p, STEP, ok, v, c);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (ok[u]) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const int q = p + u * STEP + e;
                    if (q >= beg && q < end) acc[u] = fma((double)v[u][e], (double)cl[c[u][e] - base], acc[u]);
                }
            }
    }
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// Pass 2 for operators with many rows, over the column copy in row panels of
// P rows: a work item is (panel p, a range of columns); the workgroup stages
// c's rows of panel p in LDS, then each column's segment in that panel
// (entries pp[p*n + j] .. pp[(p+1)*n + j]) is summed from LDS into
// ypanel[p*n + j].  k_pass2_panel_sum adds a column's panel sums in panel
// order and applies the column step.
template <int LPR, int VEC, typename VT>
__global__ __launch_bounds__(kLdsPassBlock) void k_pass2_panel(SpView At, const int32_t *__restrict__ pp, int np,
                                                               int P, long long m, int cpt, int chunks, int local,
                                                               const float *__restrict__ c,
                                                               double *__restrict__ ypanel,
                                                               const SliceState *__restrict__ st_in)
{
    extern __shared__ float4 cl4[];
    const float *cl = reinterpret_cast<const float *>(cl4);
    constexpr int GROUPS = kLdsPassBlock / LPR;
    if (!st_in[0].live) return; // the same in every workgroup: k_pass2_panel_sum skips the slice too
    const int lane = threadIdx.x & (LPR - 1);
    const int grp = threadIdx.x / LPR;
    const int n = (int)At.rows;
    for (int t = blockIdx.x; t < np * chunks; t += gridDim.x) {
        const int p = t / chunks, q = t % chunks;
        const long long base = (long long)p * P;
        const int len = (int)min((long long)P, m - base);
        __syncthreads(); // the previous item's readers are done with the LDS copy
        stage_vector<kLdsPassBlock>(cl4, c + base, len);
        __syncthreads();
        const int j1 = min(n, (q + 1) * cpt);
        for (int j = q * cpt + grp; j < j1; j += GROUPS) {
            const int beg = pp[(long long)p * n + j], end = pp[(long long)(p + 1) * n + j];
            const double y =
                group_sum<LPR>(seg_dot_lds<LPR, VEC, VT>(At, beg, end, lane, cl, local ? 0 : (int)base));
            if (lane == 0) ypanel[(long long)p * n + j] = y;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_pass2_panel_sum(int np, int n, const double *__restrict__ ypanel,
                                                            float vscale_inv, float *__restrict__ x, ColStep cs,
                                                            const SliceState *__restrict__ st_in,
                                                            SliceState *__restrict__ st_out,
                                                            const double *__restrict__ part1, int nparts1, Hist h)
{
    __shared__ double lds[4];
    double yacc = 0.0;
    if (st_in[0].live) {
        for (int j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock) {
            double y = 0.0;
            for (int p = 0; p < np; ++p) y += ypanel[(long long)p * n + j];
            float xo = 0.f;
            if (!cs.defer) xo = x[j];
            yacc += epi2(cs, j, j, y * (double)vscale_inv, xo, cs.lo[j], cs.hi[j], x);
        }
    }
    end_pass2(cs, yacc, st_in, st_out, part1, nparts1, h, lds);
}

template <int VEC, typename VT>
__global__ __launch_bounds__(kBlock) void k_pass2_stream(SpView At, RowBlocks RB, const float *__restrict__ c,
                                                         float *__restrict__ x, ColStep cs,
                                                         const SliceState *__restrict__ st_in,
                                                         SliceState *__restrict__ st_out,
                                                         const double *__restrict__ part1, int nparts1, Hist h)
{
    __shared__ double prod[kStreamEntries / VEC];
    __shared__ int rp[kBlock + 1];
    __shared__ double lds[4];
    double yacc = 0.0;
    if (st_in[0].live) {
        for (int b = blockIdx.x; b < RB.nblk; b += gridDim.x) {
            const int r0 = RB.rb[b], r1 = RB.rb[b + 1];
            const int e0 = At.ptr[r0], e1 = At.ptr[r1];
            if (e1 - e0 > kStreamEntries) {
                const double sum = long_row_sum<VEC, VT>(At, e0, e1, c, lds);
                if (threadIdx.x == 0)
                    yacc += epi2(cs, r0, r0, sum * (double)At.vscale_inv, x[r0], cs.lo[r0], cs.hi[r0], x);
                continue;
            }
            const int nr = r1 - r0;
            const RowSplit rs = split_rows(nr);
            const bool owner = rs.rl < nr && rs.lane == 0;
            float xo = 0.f, l = 0.f, u = 0.f;
            if (owner) {
                xo = x[r0 + rs.rl];
                l = cs.lo[r0 + rs.rl];
                u = cs.hi[r0 + rs.rl];
            }
            for (int i = threadIdx.x; i <= nr; i += kBlock) rp[i] = (At.ptr[r0 + i] - e0) / VEC;
            stream_chunks<VEC, VT>(At, e0, e1, c, prod);
            __syncthreads();
            double s = 0.0;
            if (rs.rl < nr)
                for (int q = rp[rs.rl] + rs.lane; q < rp[rs.rl + 1]; q += rs.G) s += prod[q];
            s = group_sum_rt(s, rs.G);
            if (owner) yacc += epi2(cs, r0 + rs.rl, r0 + rs.rl, s * (double)At.vscale_inv, xo, l, u, x);
            __syncthreads();
        }
    }
    end_pass2(cs, yacc, st_in, st_out, part1, nparts1, h, lds);
}

// Copies a tile's nr rows of c (B floats each, slice-interleaved as in
// memory) into LDS.  Rows are moved as float4 where B allows, and each thread
// issues U loads before its first LDS store, so that a tile's staging costs a
// few memory round trips rather than one per row a thread copies.
template <int B>
__device__ inline void stage_rows(float *__restrict__ cl, const float *__restrict__ c, const int *__restrict__ rlist,
                                  int nr)
{
    constexpr bool V4 = B % 4 == 0;
    constexpr int PER = V4 ? B / 4 : B; // loads per row
    constexpr int U = V4 ? 4 : 8;
    using V = typename std::conditional<V4, float4, float>::type;
    const int units = nr * PER;
    V *dst = reinterpret_cast<V *>(cl);
    for (int e0 = threadIdx.x; e0 < units; e0 += kBlock * U) {
        V v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) { // every load in bounds (the last unit again past the end), none predicated
            const int e = min(e0 + u * kBlock, units - 1);
            v[u] = reinterpret_cast<const V *>(c + (long long)rlist[e / PER] * B)[e % PER];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * kBlock;
            if (e < units) dst[e] = v[u];
        }
    }
}

// Pass 2 over the image-tile column layout: a workgroup takes one tile at a
// time, copies the tile's rows of c into LDS (one gather per row instead of
// one per entry: a ray crosses several pixels of a tile), then sums each
// column of the tile with LPR lanes from LDS and applies the column step.
template <int LPR, int VEC, typename VT>
__global__ __launch_bounds__(kBlock) void k_pass2_tile(TileView T, const float *__restrict__ c,
                                                       float *__restrict__ x, ColStep cs,
                                                       const SliceState *__restrict__ st_in,
                                                       SliceState *__restrict__ st_out,
                                                       const double *__restrict__ part1, int nparts1, Hist h)
{
    extern __shared__ float cl[];
    __shared__ double lds[4];
    constexpr int RPB = kBlock / LPR;
    double yacc = 0.0;
    if (st_in[0].live) {
        const int lane = threadIdx.x & (LPR - 1);
        const int grp = threadIdx.x / LPR;
        for (int t = blockIdx.x; t < T.ntiles; t += gridDim.x) {
            const int r0 = T.rptr[t], nr = T.rptr[t + 1] - r0;
            __syncthreads(); // the previous tile's readers are done with cl
            stage_rows<1>(cl, c, T.rlist + r0, nr);
            __syncthreads();
            const int p0 = T.pptr[t], np = T.pptr[t + 1] - p0;
            for (int q = grp; q < np; q += RPB) {
                const int col = T.tcol[p0 + q];
                const int beg = T.A.ptr[p0 + q], end = T.A.ptr[p0 + q + 1];
                float xo = 0.f, l = 0.f, u = 0.f;
                if (lane == 0 && !cs.defer) {
                    xo = x[col];
                    l = cs.lo[col];
                    u = cs.hi[col];
                }
                const double y = group_sum<LPR>(row_dot<LPR, VEC, VT>(T.A, beg, end, lane, cl)) * (double)T.A.vscale_inv;
                if (lane == 0) yacc += epi2(cs, col, col, y, xo, l, u, x);
            }
        }
    }
    end_pass2(cs, yacc, st_in, st_out, part1, nparts1, h, lds);
}

// ---------------------------------------------------------------------------
// Fused single pass (one slice; y = A^T c small enough to live in LDS).  The
// two passes of the feasibility step touch the same entries: row i gives r_i,
// then t_i and c_i = D_i t_i, and c_i a_i is exactly row i's contribution to
// y = A^T c.  So each workgroup streams a contiguous range of CSR rows once,
// forms c_i as pass 1 does and, while the row is still in the cache, adds
// c_i a_i into its own copy of y in LDS (float64 atomics, or float32 when a
// float64 copy does not fit).  Rows inside their band (t_i = 0) add nothing.
// The workgroup's y leaves as one partial vector; k_fused_apply sums the
// partials in workgroup order and applies x = clip(z + lambda y).  A is read
// from memory once per iteration instead of twice, and the column copy of A
// is not read at all.  Summation order inside a workgroup follows the LDS
// atomics, so results agree with the two-pass kernels up to float64 rounding.
// ---------------------------------------------------------------------------

// smallest r in [0, rows] with ptr[r] >= target (ptr[rows] >= target)
__device__ inline int first_row_at(const int *__restrict__ ptr, int rows, long long target)
{
    int lo = 0, hi = rows;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ptr[mid] >= target) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

__device__ inline void lds_add(double *a, double v) { atomicAdd(a, v); }
__device__ inline void lds_add(float *a, double v) { atomicAdd(a, (float)v); }

// y[c_j] += sc * a_ij over row [beg, end) (y in LDS), by lane `lane` of an
// LPR-lane group, the row's entries read again (from the cache) one chunk at
// a time.  Group `grp` starts at chunk grp mod (chunks of the row):
// neighbouring rows list the same columns in the same order, so the groups of
// a wave add into different words at once.  (Four chunks' loads in flight
// before their adds measured slower: 674 against 650 us on the radiotherapy
// operator, the LDS atomics rather than the loads setting the pace.)
template <int LPR, int VEC, typename VT, typename AccT>
__device__ inline void scatter_row(const SpView &A, int beg, int end, int lane, int grp, double sc, AccT *y)
{
    constexpr int STEP = LPR * VEC;
    const int nch = (end - beg + STEP - 1) / STEP;
    int q = grp % nch;
    for (int u = 0; u < nch; ++u) {
        const int p = beg + q * STEP + lane * VEC;
        if (++q == nch) q = 0;
        if (p >= end) continue;
        float v[VEC];
        int c[VEC];
        Entries<VT, VEC>::load(A, p, v, c);
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            if (v[e] != 0.f) lds_add(&y[c[e]], sc * (double)v[e]);
    }
}

template <int LPR, int VEC, typename VT, typename AccT>
__global__ __launch_bounds__(kFusedBlock) void k_fused(SpView A, int n, const float *__restrict__ x,
                                                       const float *__restrict__ lower,
                                                       const float *__restrict__ upper, RowW w,
                                                       const SliceState *__restrict__ st,
                                                       double *__restrict__ partials, AccT *__restrict__ ypart)
{
    extern __shared__ __align__(16) unsigned char fused_lds[];
    AccT *y = reinterpret_cast<AccT *>(fused_lds);
    __shared__ double lds[kFusedBlock / 64];
    __shared__ int range[2];
    constexpr int RPB = kFusedBlock / LPR;
    const int lane = threadIdx.x & (LPR - 1);
    const int grp = threadIdx.x / LPR;
    const bool live = st[0].live != 0;
    for (int j = threadIdx.x; j < n; j += kFusedBlock) y[j] = AccT(0);
    if (threadIdx.x == 0) { // an equal share of the stored entries
        const long long total = A.ptr[A.rows];
        range[0] = first_row_at(A.ptr, (int)A.rows, total * blockIdx.x / gridDim.x);
        range[1] = first_row_at(A.ptr, (int)A.rows, total * (blockIdx.x + 1) / gridDim.x);
    }
    __syncthreads();
    const int r0 = range[0], r1 = range[1];
    double pacc[1] = {0.0};
    if (live) {
        for (int row = r0 + grp; row < r1; row += RPB) {
            const int beg = A.ptr[row], end = A.ptr[row + 1];
            const float lo = lower[row], up = upper[row], d = w.D[row], sw = w.S[row];
            const double r = group_sum<LPR>(row_dot<LPR, VEC, VT>(A, beg, end, lane, x)) * (double)A.vscale_inv;
            const double t = fmin(fmax(r, (double)lo), (double)up) - r;
            const double dt = (double)d * t, ct = (double)sw * t;
            if (lane == 0) pacc[0] += dt * t;
            if (ct != 0.0 && end > beg) // the same entries again, now from the cache
                scatter_row<LPR, VEC, VT, AccT>(A, beg, end, lane, grp, ct * (double)A.vscale_inv, y);
        }
    }
    block_sum<1, kFusedBlock>(pacc, lds); // its barriers also order the LDS adds before the copy-out
    if (!live) return;
    if (threadIdx.x == 0) partials[blockIdx.x] = pacc[0];
    AccT *out = ypart + (long long)blockIdx.x * n;
    for (int j = threadIdx.x; j < n; j += kFusedBlock) out[j] = y[j];
}

// Register-cached, software-pipelined form of the fused pass.  A group of
// LPR lanes keeps up to CAP chunks (LPR*VEC entries each) of its row in
// registers, so the scatter of c_i a_i reuses the loaded entries instead of
// reading them again.  While row i is being reduced and scattered, the
// entries of the group's next row and the offsets and band of the row after
// it are already in flight.  Within a group, lane l holds the chunk slots of
// lane (l + group) mod LPR: the groups of a wave (neighbouring rows, which
// often list the same columns in the same order) then touch different
// columns in the same LDS atomic instruction, and each group still reads one
// contiguous stretch of its row.  Entries past CAP chunks (rows longer than
// CAP*LPR*VEC) are streamed and re-read from the cache as in k_fused.  Two
// rows in registers need more than the 128 registers a 1024-thread
// workgroup leaves a lane, so these workgroups have 512 threads.
template <int VEC, int CAP>
struct RowRegs {
    float v[CAP][VEC];
    int c[CAP][VEC];
};

template <int LPR, int VEC, int CAP, typename VT>
__device__ inline void fetch_entries(const SpView &A, int beg, int end, int slot, RowRegs<VEC, CAP> &R)
{
    bool ok[CAP];
#pragma unroll
    for (int q = 0; q < CAP; ++q) ok[q] = beg + (q * LPR + slot) * VEC < end;
    load_chunks<VT, VEC, CAP>(A, beg + slot * VEC, LPR * VEC, ok, R.v, R.c);
}

template <int LPR, int VEC, int CAP, typename VT, typename AccT>
__global__ __launch_bounds__(kFusedRcBlock) void k_fused_rc(SpView A, int n, const float *__restrict__ x,
                                                          const float *__restrict__ lower,
                                                          const float *__restrict__ upper, RowW w,
                                                          const SliceState *__restrict__ st,
                                                          double *__restrict__ partials, AccT *__restrict__ ypart)
{
    extern __shared__ __align__(16) unsigned char fused_lds[];
    AccT *y = reinterpret_cast<AccT *>(fused_lds);
    __shared__ double lds[kFusedRcBlock / 64];
    __shared__ int range[2];
    constexpr int RPB = kFusedRcBlock / LPR;
    constexpr int STEP = LPR * VEC;
    const int lane = threadIdx.x & (LPR - 1);
    const int grp = threadIdx.x / LPR;
    const int slot = (lane + grp) & (LPR - 1);
    const bool live = st[0].live != 0;
    for (int j = threadIdx.x; j < n; j += kFusedRcBlock) y[j] = AccT(0);
    if (threadIdx.x == 0) {
        const long long total = A.ptr[A.rows];
        range[0] = first_row_at(A.ptr, (int)A.rows, total * blockIdx.x / gridDim.x);
        range[1] = first_row_at(A.ptr, (int)A.rows, total * (blockIdx.x + 1) / gridDim.x);
    }
    __syncthreads();
    const int r0 = range[0], r1 = range[1];
    double pacc[1] = {0.0};
    int row = r0 + grp;
    if (live && row < r1) {
        // row `row`: entries in cur; row + RPB: offsets/band in nb..; entries follow
        RowRegs<VEC, CAP> cur, nxt;
        int beg = A.ptr[row], end = A.ptr[row + 1];
        float lo = lower[row], up = upper[row], d = w.D[row], sw = w.S[row];
        fetch_entries<LPR, VEC, CAP, VT>(A, beg, end, slot, cur);
        int nb = 0, ne = 0;
        float nlo = 0.f, nup = 0.f, nd = 0.f, nsw = 0.f;
        if (row + RPB < r1) {
            nb = A.ptr[row + RPB];
            ne = A.ptr[row + RPB + 1];
            nlo = lower[row + RPB];
            nup = upper[row + RPB];
            nd = w.D[row + RPB];
            nsw = w.S[row + RPB];
        }
        for (;;) {
            float xg[CAP][VEC];
#pragma unroll
            for (int q = 0; q < CAP; ++q)
#pragma unroll
                for (int e = 0; e < VEC; ++e) xg[q][e] = x[cur.c[q][e]];
            const int rn = row + RPB, rnn = row + 2 * RPB;
            if (rn < r1) fetch_entries<LPR, VEC, CAP, VT>(A, nb, ne, slot, nxt);
            int hb = 0, he = 0;
            float hlo = 0.f, hup = 0.f, hd = 0.f, hsw = 0.f;
            if (rnn < r1) {
                hb = A.ptr[rnn];
                he = A.ptr[rnn + 1];
                hlo = lower[rnn];
                hup = upper[rnn];
                hd = w.D[rnn];
                hsw = w.S[rnn];
            }
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < CAP; ++q)
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc = fma((double)cur.v[q][e], (double)xg[q][e], acc);
            const bool tail = end - beg > CAP * STEP;
            if (tail) acc += row_dot<LPR, VEC, VT>(A, beg + CAP * STEP, end, lane, x);
            const double r = group_sum<LPR>(acc) * (double)A.vscale_inv;
            const double t = fmin(fmax(r, (double)lo), (double)up) - r;
            const double dt = (double)d * t, ct = (double)sw * t;
            if (lane == 0) pacc[0] += dt * t;
            if (ct != 0.0) {
                const double sc = ct * (double)A.vscale_inv;
#pragma unroll
                for (int q = 0; q < CAP; ++q)
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        if (cur.v[q][e] != 0.f) lds_add(&y[cur.c[q][e]], sc * (double)cur.v[q][e]);
                if (tail) {
                    for (int p = beg + CAP * STEP + lane * VEC; p < end; p += STEP) {
                        float v[VEC];
                        int c[VEC];
                        Entries<VT, VEC>::load(A, p, v, c);
#pragma unroll
                        for (int e = 0; e < VEC; ++e)
                            if (v[e] != 0.f) lds_add(&y[c[e]], sc * (double)v[e]);
                    }
                }
            }
            if (rn >= r1) break;
            row = rn;
            beg = nb;
            end = ne;
            lo = nlo;
            up = nup;
            d = nd;
            sw = nsw;
            cur = nxt;
            nb = hb;
            ne = he;
            nlo = hlo;
            nup = hup;
            nd = hd;
            nsw = hsw;
        }
    }
    block_sum<1, kFusedRcBlock>(pacc, lds); // its barriers also order the LDS adds before the copy-out
    if (!live) return;
    if (threadIdx.x == 0) partials[blockIdx.x] = pacc[0];
    AccT *out = ypart + (long long)blockIdx.x * n;
    for (int j = threadIdx.x; j < n; j += kFusedRcBlock) out[j] = y[j];
}

// Direction partials of the linear objective f = c^T x for the next
// perturbation phase: this workgroup's sums of c_j^2 and c_j x_j over the
// unknowns j0 + l (l < 64, j0 = 64 blockIdx.x, stepping 64 gridDim.x),
// added by the first wave's lanes in that order and then over the
// workgroup, stored as the direction launch's partials would be (slot
// blockIdx.x of 2 x gridDim.x).  k_fused_apply calls it after writing x and
// k_lin_partials alone, with the same sums in the same order.
__device__ inline void lin_partials_block(const float *__restrict__ x, const float *__restrict__ c, int n,
                                          double *__restrict__ part, double *lds)
{
    double v[2] = {0.0, 0.0}; // sum c^2, c^T x
    if ((threadIdx.x >> 6) == 0)
        for (int j = blockIdx.x * 64 + (int)threadIdx.x; j < n; j += gridDim.x * 64) {
            const double cj = (double)c[j];
            v[0] += cj * cj;
            v[1] += cj * (double)x[j];
        }
    block_sum<2, kApplyBlock>(v, lds);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = v[0];
        part[gridDim.x + blockIdx.x] = v[1];
    }
}

__global__ __launch_bounds__(kApplyBlock) void k_lin_partials(const float *__restrict__ x,
                                                              const float *__restrict__ c, int n,
                                                              double *__restrict__ part)
{
    __shared__ double lds[kApplyBlock / 64 * 2];
    lin_partials_block(x, c, n, part, lds);
}

// x = clip(z + lambda * Z_j * sum_g ypart[g], lo, hi) (Z_j = 1 unless DROP);
// 64 unknowns per workgroup, the four waves each sum every fourth partial
// (loads issued four at a time, added in order) and the four sums are added in
// a fixed order.  Workgroup 0 also closes the outer iteration.
template <typename AccT>
__global__ __launch_bounds__(kApplyBlock) void k_fused_apply(const AccT *__restrict__ ypart, int G, int n,
                                                        float *__restrict__ x, ColStep cs,
                                                        const SliceState *__restrict__ st_in,
                                                        SliceState *__restrict__ st_out,
                                                        const double *__restrict__ part1, int nparts1, Hist h,
                                                        const float *__restrict__ lin_c, double *__restrict__ lin_part,
                                                        int lin_z)
{
    __shared__ double red[kApplyBlock / 64][64];
    __shared__ double lds[kApplyBlock / 64 * 2];
    const int wid = threadIdx.x >> 6, wl = threadIdx.x & 63;
    double ysq = 0.0; // deferred mode: this thread's share of ||y||^2
    // the linear phase taken in the pass: x still holds x^k, z_j is formed here
    bool zstep = false;
    double zs = 0.0, zinv = 0.0;
    if (lin_z && st_in[0].applied && st_in[0].s_acc != 0.0) {
        zstep = true;
        zs = st_in[0].s_acc;
        zinv = 1.0 / st_in[0].gn;
    }
    if (st_in[0].live) {
        for (int j0 = blockIdx.x * 64; j0 < n; j0 += gridDim.x * 64) {
            const int j = j0 + wl;
            constexpr int W = kApplyBlock / 64;
            double sum = 0.0;
            if (j < n) { // wave w adds partials w, w + W, ... (eight loads in flight)
                int g = wid;
                for (; g + 7 * W < G; g += 8 * W) {
                    double v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) v[u] = (double)ypart[(long long)(g + u * W) * n + j];
#pragma unroll
                    for (int u = 0; u < 8; ++u) sum += v[u];
                }
                for (; g < G; g += W) sum += (double)ypart[(long long)g * n + j];
            }
            red[wid][wl] = sum;
            __syncthreads();
            if (wid == 0 && j < n) {
                double yv = 0.0;
#pragma unroll
                for (int w = 0; w < W; ++w) yv += red[w][wl];
                if (cs.defer) { // the extrapolated steps: keep y, x moves in k_step_apply
                    cs.ybuf[j] = yv;
                    if (cs.ybuf32) cs.ybuf32[j] = (float)yv;
                    ysq += yv * yv;
                } else {
                    if (cs.zcol) yv *= (double)cs.zcol[j];
                    const float zj = zstep ? linear_step_point(x[j], lin_c[j], zs, zinv) : x[j];
                    const double z = fma((double)cs.lambda, yv, (double)zj);
                    x[j] = (float)fmin(fmax(z, (double)cs.lo[j]), (double)cs.hi[j]);
                }
            }
            __syncthreads();
        }
    }
    // the next phase's direction partials from the x just written (each
    // lane rereads its own entries)
    if (lin_part) lin_partials_block(x, lin_c, n, lin_part, lds);
    if (cs.defer) {
        double v[1] = {ysq};
        block_sum<1, kApplyBlock>(v, lds);
        if (threadIdx.x == 0) cs.ypart[blockIdx.x] = v[0];
    } else if (blockIdx.x == 0) {
        finish_iteration<kApplyBlock>(st_in, st_out, 1, part1, nparts1, h, lds);
    }
}

// Extrapolated steps (one launch after pass 2, or after the quadratic-form
// pass): per slice, sigma from the totals of the partials, each summed in
// workgroup order by every workgroup (EL: t^T D t / ||y||^2, with t^T D t
// twice pass 1's proximity sum; EMR: ||y||^2 / sum_i w_i (A y)_i^2), 0 when the
// denominator is 0 or the quotient is not finite; then
// x = clip(z + lambda sigma y, lo, hi).  Workgroup 0 also closes the iteration.
__global__ __launch_bounds__(kBlock) void k_step_apply(int n, int B, const double *__restrict__ y,
                                                       float *__restrict__ x, const float *__restrict__ lo,
                                                       const float *__restrict__ hi, float lambda, int emr,
                                                       const double *__restrict__ part1, int nparts1,
                                                       const double *__restrict__ party, int npartsy,
                                                       const double *__restrict__ partq, int npartsq,
                                                       const SliceState *__restrict__ st_in,
                                                       SliceState *__restrict__ st_out, Hist h)
{
    __shared__ double lds[4];
    __shared__ double sigma[32];
    __shared__ int live[32];
    for (int s = 0; s < B; ++s) {
        double num[1], den[1];
        if (emr) {
            sum_slots<1>(party, (long long)s * npartsy, npartsy, num, lds);
            sum_slots<1>(partq, (long long)s * npartsq, npartsq, den, lds);
        } else {
            sum_slots<1>(part1, (long long)s * nparts1, nparts1, num, lds);
            sum_slots<1>(party, (long long)s * npartsy, npartsy, den, lds);
        }
        if (threadIdx.x == 0) {
            const double q = num[0] / den[0];
            sigma[s] = (den[0] > 0.0 && isfinite(q)) ? q : 0.0;
            live[s] = st_in[s].live;
        }
    }
    __syncthreads();
    const long long total = (long long)n * B;
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < total; e += (long long)gridDim.x * kBlock) {
        const int s = (int)(e % B);
        if (!live[s]) continue;
        const long long j = e / B;
        const double z = fma((double)lambda * sigma[s], y[e], (double)x[e]);
        x[e] = (float)fmin(fmax(z, (double)lo[j]), (double)hi[j]);
    }
    if (blockIdx.x == 0) finish_iteration(st_in, st_out, B, part1, nparts1, h, lds);
}

// ---------------------------------------------------------------------------
// Multi-slice passes (B right-hand sides sharing A, slice-interleaved
// vectors).  A is read once for all slices; each lane keeps one float64
// accumulator per slice and reads the B values of the gathered vector at an
// index as B/4 vector loads.  The summation order of a slice does not depend
// on the other slices, so a slice's result is the same whichever slices run
// beside it.  A slice that is not live is neither read back nor written.
// ---------------------------------------------------------------------------

template <int B>
__device__ inline void load_slices(const float *__restrict__ v, int idx, float (&out)[B])
{
    if constexpr (B % 4 == 0) {
        const float4 *q = reinterpret_cast<const float4 *>(v + (long long)idx * B);
#pragma unroll
        for (int h = 0; h < B / 4; ++h) {
            const float4 a = q[h];
            out[4 * h + 0] = a.x; out[4 * h + 1] = a.y; out[4 * h + 2] = a.z; out[4 * h + 3] = a.w;
        }
    } else if constexpr (B == 2) {
        const float2 a = *reinterpret_cast<const float2 *>(v + (long long)idx * 2);
        out[0] = a.x; out[1] = a.y;
    } else {
#pragma unroll
        for (int s = 0; s < B; ++s) out[s] = v[(long long)idx * B + s];
    }
}

template <int LPR, int VEC, typename VT, int B>
__device__ inline void row_dot_mm(const SpView &A, int beg, int end, int lane, const float *__restrict__ v,
                                  double (&acc)[B])
{
#pragma unroll
    for (int s = 0; s < B; ++s) acc[s] = 0.0;
    for (int p = beg + lane * VEC; p < end; p += LPR * VEC) {
        float val[VEC];
        int id[VEC];
        Entries<VT, VEC>::load(A, p, val, id);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            float xs[B];
            load_slices<B>(v, id[e], xs);
            const double a = (double)val[e];
#pragma unroll
            for (int s = 0; s < B; ++s) acc[s] = fma(a, (double)xs[s], acc[s]);
        }
    }
#pragma unroll
    for (int s = 0; s < B; ++s) acc[s] = group_sum<LPR>(acc[s]);
}

template <int LPR, int VEC, typename VT, int B>
__global__ __launch_bounds__(kBlock) void k_pass1_mm(SpView A, const float *__restrict__ x,
                                                     const float *__restrict__ lower, const float *__restrict__ upper,
                                                     RowW w, float *__restrict__ c,
                                                     const SliceState *__restrict__ st, int query,
                                                     double *__restrict__ partials)
{
    __shared__ double lds[4 * B];
    __shared__ int live[B];
    constexpr int RPB = kBlock / LPR;
    if (threadIdx.x < B) live[threadIdx.x] = query ? 1 : st[threadIdx.x].live;
    __syncthreads();
    const int lane = threadIdx.x & (LPR - 1);
    const int grp = threadIdx.x / LPR;
    double pacc[B];
#pragma unroll
    for (int s = 0; s < B; ++s) pacc[s] = 0.0;
    const long long stride = (long long)gridDim.x * RPB;
    for (long long row = (long long)blockIdx.x * RPB + grp; row < A.rows; row += stride) {
        const int beg = A.ptr[row], end = A.ptr[row + 1];
        double acc[B];
        row_dot_mm<LPR, VEC, VT, B>(A, beg, end, lane, x, acc);
        if (lane == 0) {
            const float d = w.D[row], sw = w.S[row];
#pragma unroll
            for (int s = 0; s < B; ++s) {
                if (!live[s]) continue;
                pacc[s] += epi1(w, acc[s] * (double)A.vscale_inv, lower[row * B + s], upper[row * B + s], d, sw,
                                c + row * B + s, row, s, B);
            }
        }
    }
    block_sum<B>(pacc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int s = 0; s < B; ++s) partials[(long long)s * gridDim.x + blockIdx.x] = pacc[s];
    }
}

template <int LPR, int VEC, typename VT, int B>
__global__ __launch_bounds__(kBlock) void k_pass2_mm(SpView At, const float *__restrict__ c, float *__restrict__ x,
                                                     ColStep cs, const SliceState *__restrict__ st_in,
                                                     SliceState *__restrict__ st_out,
                                                     const double *__restrict__ part1, int nparts1, Hist h)
{
    __shared__ double lds[4 * B];
    __shared__ int live[B];
    constexpr int RPB = kBlock / LPR;
    if (threadIdx.x < B) live[threadIdx.x] = st_in[threadIdx.x].live;
    __syncthreads();
    const int lane = threadIdx.x & (LPR - 1);
    const int grp = threadIdx.x / LPR;
    double yacc[B];
#pragma unroll
    for (int s = 0; s < B; ++s) yacc[s] = 0.0;
    const long long stride = (long long)gridDim.x * RPB;
    for (long long col = (long long)blockIdx.x * RPB + grp; col < At.rows; col += stride) {
        const int beg = At.ptr[col], end = At.ptr[col + 1];
        double acc[B];
        row_dot_mm<LPR, VEC, VT, B>(At, beg, end, lane, c, acc);
        if (lane == 0) {
            const float l = cs.lo[col], u = cs.hi[col];
#pragma unroll
            for (int s = 0; s < B; ++s) {
                if (!live[s]) continue;
                yacc[s] += epi2(cs, col, col * B + s, acc[s] * (double)At.vscale_inv, x[col * B + s], l, u, x);
            }
        }
    }
    if (cs.defer) {
        block_sum<B>(yacc, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int s = 0; s < B; ++s) cs.ypart[(long long)s * gridDim.x + blockIdx.x] = yacc[s];
        }
    } else if (blockIdx.x == 0) {
        finish_iteration(st_in, st_out, B, part1, nparts1, h, lds);
    }
}

// Pass 2 over the image-tile column layout for B slices: the tile's rows of
// c (B values each, slice-interleaved as in memory) are staged in LDS, and
// every entry of a column reads its B values from there, as k_pass2_tile does
// for one slice.  Each slice's sums follow the same order as in k_pass2_tile.
template <int LPR, int VEC, typename VT, int B>
__global__ __launch_bounds__(kBlock) void k_pass2_tile_mm(TileView T, const float *__restrict__ c,
                                                          float *__restrict__ x, ColStep cs,
                                                          const SliceState *__restrict__ st_in,
                                                          SliceState *__restrict__ st_out,
                                                          const double *__restrict__ part1, int nparts1, Hist h)
{
    extern __shared__ float4 cl4[]; // 16-byte aligned: rows of B floats
    float *cl = reinterpret_cast<float *>(cl4);
    __shared__ double lds[4 * B];
    __shared__ int live[B];
    constexpr int RPB = kBlock / LPR;
    if (threadIdx.x < B) live[threadIdx.x] = st_in[threadIdx.x].live;
    __syncthreads();
    bool any = false;
#pragma unroll
    for (int s = 0; s < B; ++s) any = any || live[s];
    const int lane = threadIdx.x & (LPR - 1);
    const int grp = threadIdx.x / LPR;
    double yacc[B];
#pragma unroll
    for (int s = 0; s < B; ++s) yacc[s] = 0.0;
    if (any) {
        for (int t = blockIdx.x; t < T.ntiles; t += gridDim.x) {
            const int r0 = T.rptr[t], nr = T.rptr[t + 1] - r0;
            __syncthreads(); // the previous tile's readers are done with cl
            stage_rows<B>(cl, c, T.rlist + r0, nr);
            __syncthreads();
            const int p0 = T.pptr[t], np = T.pptr[t + 1] - p0;
            for (int q = grp; q < np; q += RPB) {
                const int col = T.tcol[p0 + q];
                const int beg = T.A.ptr[p0 + q], end = T.A.ptr[p0 + q + 1];
                double acc[B];
                row_dot_mm<LPR, VEC, VT, B>(T.A, beg, end, lane, cl, acc);
                if (lane == 0) {
                    const float l = cs.lo[col], u = cs.hi[col];
#pragma unroll
                    for (int s = 0; s < B; ++s) {
                        if (!live[s]) continue;
                        yacc[s] += epi2(cs, col, (long long)col * B + s, acc[s] * (double)T.A.vscale_inv,
                                        x[(long long)col * B + s], l, u, x);
                    }
                }
            }
        }
    }
    if (cs.defer) {
        block_sum<B>(yacc, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int s = 0; s < B; ++s) cs.ypart[(long long)s * gridDim.x + blockIdx.x] = yacc[s];
        }
    } else if (blockIdx.x == 0) {
        finish_iteration(st_in, st_out, B, part1, nparts1, h, lds);
    }
}

// Query: the proximity at the current x from pass 1's partials (query mode).
__global__ __launch_bounds__(kBlock) void k_query_prox(SliceState *__restrict__ st, int B,
                                                       const double *__restrict__ partials, int nparts,
                                                       double *__restrict__ out)
{
    __shared__ double lds[4];
    for (int s = 0; s < B; ++s) {
        double tot[1];
        sum_slots<1>(partials, (long long)s * nparts, nparts, tot, lds);
        if (threadIdx.x == 0) {
            out[s] = 0.5 * tot[0];
            if (!isfinite(out[s])) st[s].nonfinite = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// perturbation phase
//
// Launch sequence of one phase: gradient (partials of ||g||^2 and f(x^k) per
// tile), then trial launches, then a closing launch.  Each trial launch first
// re-derives, in every workgroup, what the previous launch decided (the first
// launch: the opening of the phase) from that launch's partials, then either
// evaluates the next batch of trial steps or, once the phase is over, adds the
// accepted step s_acc v to its own tile of x.  Partials are stored value-major
// ([value][slice*tiles + tile]) so the re-derivation reads them coalesced.
// ---------------------------------------------------------------------------

// Step of trial e (the trial exponent): the power law gamma alpha^e, or the
// phase's adaptive step (Section 2.1.2), the same for its one trial.
__device__ inline double trial_beta(const PertParams &pp, const SliceState &S, long long e)
{
    return pp.adaptive ? S.beta_ad : pp.gamma * pow(pp.alpha, (double)e);
}

// Number of trials a trial launch evaluates for slice state S: a short batch
// when a reduction step starts, all remaining ones (up to the cap) after that.
// Trials a launch evaluates: the first batch of a reduction step is the
// default width, widened to 1.5x the trials the previous step needed (step
// sizes shrink along the phase, so that is usually enough); a second batch
// takes every trial left up to the cap.  The width only decides how many
// trials are evaluated speculatively: the accepted trial is the first
// acceptable one in order whatever the width.
__device__ inline int trial_width(const SliceState &S, const PertParams &pp)
{
    if (!S.phase) return 0;
    const int left = pp.max_trials - S.step_tried;
    if (S.step_tried != 0) return left;
    int w = pp.first_width;
    const int want = S.need_last + (S.need_last >> 1);
    if (want > w) w = ((want + kFirstWidth - 1) / kFirstWidth) * kFirstWidth;
    return min(w, left);
}

// Grid of the phase kernels: blockIdx.y is the slice, blockIdx.x a tile (TV)
// or a chunk of the vector.
int phase_grid(const PertParams &pp)
{
    if (pp.obj == OBJ_TV2D) return ((pp.tv_rows + kTile - 1) / kTile) * ((pp.tv_cols + kTile - 1) / kTile);
    long long g = (pp.n + kBlock * 4 - 1) / (kBlock * 4);
    return (int)(g < 1 ? 1 : (g > 512 ? 512 : g));
}

// Totals over the `nt` tiles of slice s of rows v0 .. v0+nv-1 (rows of
// `nslots` slots, nv <= kTrialChunk) into tot[0..nv-1] (LDS), for a workgroup
// of BS threads; every thread must call it, and tot is valid for every thread
// on return.  Row v0+r is summed by wave r mod (BS/64): lane l adds tiles
// l, l+64, ... in order, then the lanes are added by wave_sum.  The rows of a
// wave, and U tiles of each, are loaded together, so their loads overlap.
template <int BS>
__device__ inline void chunk_totals(const double *__restrict__ part, long long nslots, int s, int nt, int v0, int nv,
                                    double *tot)
{
    constexpr int W = BS / 64, RPW = (kTrialChunk + W - 1) / W;
    constexpr int U = RPW >= 16 ? 1 : 16 / RPW;
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double a[RPW];
#pragma unroll
    for (int q = 0; q < RPW; ++q) a[q] = 0.0;
    if (wid < nv) {
        for (int b0 = lane; b0 < nt; b0 += 64 * U) {
            double v[U][RPW];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int b = min(b0 + 64 * u, nt - 1); // past nt: loaded, not added
#pragma unroll
                for (int q = 0; q < RPW; ++q)
                    v[u][q] = part[(long long)(v0 + min(wid + W * q, nv - 1)) * nslots + (long long)s * nt + b];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (b0 + 64 * u < nt) {
#pragma unroll
                    for (int q = 0; q < RPW; ++q) a[q] += v[u][q];
                }
        }
        wave_sum<RPW>(a);
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < RPW; ++q)
                if (wid + W * q < nv) tot[wid + W * q] = a[q];
        }
    }
    __syncthreads();
}

// Opening of a phase from the totals (sum g^2, f(x^k)).
__device__ inline void open_phase_state(SliceState &S, const PertParams &pp, double gsq, double f)
{
    S.trials_it = 0;
    S.accepts_it = 0;
    S.s_acc = 0.0;
    S.n_done = 0;
    S.step_tried = 0;
    S.applied = 0;
    if (!S.live) {
        S.phase = 0;
        S.f_start = S.f_cur = nan64();
        return;
    }
    // superiorized stopping rule (Section 2.2.3): a proximity rule held at the
    // last iteration and |f(x^k) - f(x^{k-1})| / max{1, f(x^{k-1})} < Delta f*
    if (S.stop_on && S.feas_ok && !isnan(S.f_last) && fabs(f - S.f_last) / fmax(1.0, S.f_last) < S.stop_dobj) {
        S.stop_reason = STOP_SM;
        S.live = 0;
        S.phase = 0;
        S.f_start = S.f_cur = nan64();
        return;
    }
    if (pp.restart_every > 0 && S.k > 0 && (S.k % pp.restart_every) == 0) {
        S.restarts += 1;
        S.ell = S.restarts;
    }
    S.gn = sqrt(gsq);
    S.f_start = S.f_cur = f;
    if (!isfinite(f) || !isfinite(S.gn)) S.nonfinite = 1;
    S.phase = (S.gn > 0.0 && isfinite(S.gn)) ? 1 : 0;
    if (pp.adaptive) { // one step to the reference value, none before there is one or when f is at or below it
        if (S.phase && !isnan(S.f_ref) && f > S.f_ref) S.beta_ad = (f - S.f_ref) / S.gn;
        else S.phase = 0;
    }
}

// The state after a batch of ntr trials (steps ell .. ell+ntr-1 of the power
// law, or the one adaptive step) was evaluated: acc_t is the first trial in
// order whose objective does not exceed f_cur (-1 when none does), acc_f its
// objective.  Accepting ends the reduction step (and the phase after n_red of
// them); a step that reaches the trial cap unaccepted ends the phase.
__device__ inline void record_decision(SliceState &S, const PertParams &pp, int ntr, int acc_t, double acc_f)
{
    if (acc_t >= 0) {
        S.s_acc = S.s_acc + trial_beta(pp, S, S.ell + acc_t);
        S.f_cur = acc_f;
        if (!isfinite(acc_f)) S.nonfinite = 1;
        S.ell += acc_t + 1;
        S.trials_it += acc_t + 1;
        S.trials += acc_t + 1;
        S.accepts_it += 1;
        S.accepts += 1;
        S.n_done += 1;
        S.need_last = S.step_tried + acc_t + 1;
        S.step_tried = 0;
        if (S.n_done >= pp.n_red) S.phase = 0;
    } else {
        S.ell += ntr;
        S.trials_it += ntr;
        S.trials += ntr;
        S.step_tried += ntr;
        if (S.step_tried >= pp.max_trials) {
            if (!pp.adaptive) S.cap_hits += 1; // a rejected adaptive step simply ends the phase
            S.need_last = pp.max_trials;
            S.phase = 0;
        }
    }
}

// Every workgroup: the state after the previous trial launch of slice s, in
// sS (LDS).  The first trial in order whose objective does not exceed f_cur is
// accepted; reading stops at the chunk holding it.
template <int BS>
__device__ inline void derive_decision(SliceState &sS, const PertParams &pp, const double *__restrict__ part_prev,
                                       long long nslots, int s, int nt, double *tot)
{
    __shared__ int acc_t;
    __shared__ double acc_f;
    const int ntr = trial_width(sS, pp);
    if (ntr == 0) return;
    if (threadIdx.x == 0) acc_t = -1;
    for (int t0 = 0; t0 < ntr; t0 += kTrialChunk) {
        const int nv = min(kTrialChunk, ntr - t0);
        chunk_totals<BS>(part_prev, nslots, s, nt, t0, nv, tot);
        if (threadIdx.x == 0) {
            for (int w = 0; w < nv; ++w) {
                if (tot[w] <= sS.f_cur) {
                    acc_t = t0 + w;
                    acc_f = tot[w];
                    break;
                }
            }
        }
        __syncthreads();
        if (acc_t >= 0) break;
    }
    if (threadIdx.x == 0) record_decision(sS, pp, ntr, acc_t, acc_f);
    __syncthreads();
}

// Every workgroup: state of slice s at the start of this launch, in sS.
// mode 0: the first trial launch (opens the phase from the gradient partials);
// otherwise: the decision of the previous trial launch.
template <int BS>
__device__ inline void derive_state(SliceState &sS, const SliceState *__restrict__ st_in, const PertParams &pp,
                                    int first, const double *__restrict__ part_prev, int s, int nt, double *tot)
{
    if (threadIdx.x == 0) sS = st_in[s];
    const long long nslots = (long long)pp.B * nt;
    if (first) { // the state's loads overlap the partials' (thread 0 alone reads sS before the barriers)
        chunk_totals<BS>(part_prev, nslots, s, nt, 0, 2, tot);
        if (threadIdx.x == 0) open_phase_state(sS, pp, tot[0], tot[1]);
        __syncthreads();
    } else {
        __syncthreads();
        derive_decision<BS>(sS, pp, part_prev, nslots, s, nt, tot);
    }
}

__device__ inline void publish_state(const SliceState &S, SliceState *__restrict__ st_out, int s, bool applied_here)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        SliceState o = S;
        if (applied_here) o.applied = 1;
        st_out[s] = o;
    }
}

// Whether this launch adds the accepted step to x (the phase is over).
__device__ inline bool must_apply(const SliceState &S) { return S.live && !S.phase && !S.applied && S.s_acc != 0.0; }

// -- TV2D: smoothed total variation on an R x C image, pixel (i,j) = unknown i*C + j.
//    Terms at (i,j) for i <= R-2, j <= C-2: tau = sqrt(dx^2 + dy^2 + eps^2) with
//    dx = X[i+1,j] - X[i,j], dy = X[i,j+1] - X[i,j].

__device__ inline double tv_tau(double x00, double x10, double x01, double eps2)
{
    const double dx = x10 - x00, dy = x01 - x00;
    return sqrt(dx * dx + dy * dy + eps2);
}

// Gradient (unless eval_only) and per-tile partials of ||g||^2 and f(x); the
// tile carries a one-pixel halo on every side.
__global__ __launch_bounds__(kBlock) void k_phase_tv(const float *__restrict__ x, float *__restrict__ g,
                                                     const SliceState *__restrict__ st, PertParams pp, int eval_only,
                                                     double *__restrict__ partials)
{
    __shared__ float tile[kTile + 2][kTile + 3];
    __shared__ double lds[4 * 2];
    const int s = blockIdx.y, B = pp.B;
    const int R = pp.tv_rows, C = pp.tv_cols;
    const int tiles_x = (C + kTile - 1) / kTile;
    const int i0 = (blockIdx.x / tiles_x) * kTile, j0 = (blockIdx.x % tiles_x) * kTile;
    const bool live = eval_only ? true : st[s].live != 0;
    double v[2] = {0.0, 0.0}; // sum g^2, f
    if (live) {
        for (int e = threadIdx.x; e < (kTile + 2) * (kTile + 2); e += kBlock) {
            const int li = e / (kTile + 2), lj = e % (kTile + 2);
            const int gi = i0 - 1 + li, gj = j0 - 1 + lj;
            float val = 0.f;
            if (gi >= 0 && gi < R && gj >= 0 && gj < C) val = x[((long long)gi * C + gj) * B + s];
            tile[li][lj] = val;
        }
        __syncthreads();
        const int li = threadIdx.x / kTile, lj = threadIdx.x % kTile;
        const int i = i0 + li, j = j0 + lj;
        if (i < R && j < C) {
#define XT(a, b) ((double)tile[(a) - i0 + 1][(b) - j0 + 1])
            double gv = 0.0;
            if (i <= R - 2 && j <= C - 2) {
                const double x00 = XT(i, j), x10 = XT(i + 1, j), x01 = XT(i, j + 1);
                const double tau = tv_tau(x00, x10, x01, pp.tv_eps2);
                v[1] = tau;
                if (tau > 0.0) gv -= ((x10 - x00) + (x01 - x00)) / tau;
            }
            if (i >= 1 && j <= C - 2) { // term (i-1, j): this pixel is its +1 row neighbour
                const double x00 = XT(i - 1, j), x10 = XT(i, j), x01 = XT(i - 1, j + 1);
                const double tau = tv_tau(x00, x10, x01, pp.tv_eps2);
                if (tau > 0.0) gv += (x10 - x00) / tau;
            }
            if (j >= 1 && i <= R - 2) { // term (i, j-1): this pixel is its +1 column neighbour
                const double x00 = XT(i, j - 1), x10 = XT(i + 1, j - 1), x01 = XT(i, j);
                const double tau = tv_tau(x00, x10, x01, pp.tv_eps2);
                if (tau > 0.0) gv += (x01 - x00) / tau;
            }
#undef XT
            if (!eval_only) {
                const float gf = (float)gv;
                g[((long long)i * C + j) * B + s] = gf;
                v[0] = (double)gf * (double)gf;
            }
        }
    }
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        const long long nslots = (long long)gridDim.x * gridDim.y, slot = (long long)s * gridDim.x + blockIdx.x;
        partials[slot] = v[0];
        partials[nslots + slot] = v[1];
    }
}

// Squared norm (g = 2x), L1 norm (g = sign x) and linear objective (g = c) versions.
__global__ __launch_bounds__(kBlock) void k_phase_flat(const float *__restrict__ x, float *__restrict__ g,
                                                       const float *__restrict__ lin_c,
                                                       const SliceState *__restrict__ st, PertParams pp,
                                                       int eval_only, double *__restrict__ partials)
{
    __shared__ double lds[4 * 2];
    const int s = blockIdx.y, B = pp.B;
    const bool live = eval_only ? true : st[s].live != 0;
    double v[2] = {0.0, 0.0};
    if (live) {
        for (long long j = (long long)blockIdx.x * kBlock + threadIdx.x; j < pp.n; j += (long long)gridDim.x * kBlock) {
            const double xj = (double)x[j * B + s];
            if (pp.obj == OBJ_SQNORM) {
                v[1] += xj * xj;
                if (!eval_only) {
                    const float gf = (float)(2.0 * xj);
                    g[j * B + s] = gf;
                    v[0] += (double)gf * (double)gf;
                }
            } else if (pp.obj == OBJ_L1) { // subgradient sign(x), 0 at 0
                v[1] += fabs(xj);
                if (!eval_only) {
                    const float gf = xj > 0.0 ? 1.f : (xj < 0.0 ? -1.f : 0.f);
                    g[j * B + s] = gf;
                    v[0] += (double)gf * (double)gf;
                }
            } else { // OBJ_LINEAR
                const double cj = (double)lin_c[j];
                v[1] += cj * xj;
                v[0] += cj * cj;
            }
        }
    }
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        const long long nslots = (long long)gridDim.x * gridDim.y, slot = (long long)s * gridDim.x + blockIdx.x;
        partials[slot] = v[0];
        partials[nslots + slot] = v[1];
    }
}

// Objective per slice from k_phase_* partials in eval_only mode (one workgroup).
__global__ __launch_bounds__(kBlock) void k_eval_objective(SliceState *__restrict__ st, PertParams pp,
                                                           const double *__restrict__ partials, int nt,
                                                           double *__restrict__ out)
{
    __shared__ double tot[kTrialChunk];
    for (int s = 0; s < pp.B; ++s) {
        chunk_totals<kBlock>(partials, (long long)pp.B * nt, s, nt, 0, 2, tot);
        if (threadIdx.x == 0) {
            out[s] = tot[1];
            if (!isfinite(tot[1])) st[s].nonfinite = 1;
        }
        __syncthreads();
    }
}

// Trial launch for TV (kTrialBlock threads per 16 x 16 tile): derive the
// state, then evaluate tau at z = x + (s_acc + beta_t) v for every trial t of
// this launch and every pixel term of the tile (one partial per trial per
// tile); or, once the phase is over, add s_acc v to the tile.  Wave w takes
// trials w*4 .. w*4+3, then the next 4 * (waves) trials, and so on; lane l of a
// wave takes pixels l, l+64, l+128, l+192 of the tile, adds its terms in that
// order, and wave_sum adds the lanes: each trial's tile sum is made by one
// wave, with no workgroup barrier, and the 16 waves keep the float64 square
// roots of different trials in flight together.
__global__ __launch_bounds__(kTrialBlock) void k_trial_tv(float *__restrict__ x, const float *__restrict__ g,
                                                          const SliceState *__restrict__ st_in,
                                                          SliceState *__restrict__ st_out, PertParams pp, int first,
                                                          int evaluate, const double *__restrict__ part_prev,
                                                          double *__restrict__ part_out)
{
    static_assert(kTile * kTile == 256, "tile of 256 pixels");
    __shared__ float tx[kTile + 1][kTile + 2];
    __shared__ float tg[kTile + 1][kTile + 2];
    __shared__ double coef[1024];
    __shared__ double tot[kTrialChunk];
    __shared__ SliceState sS;
    constexpr int W = kTrialBlock / 64;
    const int s = blockIdx.y, B = pp.B, nt = gridDim.x;
    const int R = pp.tv_rows, C = pp.tv_cols;
    const int tiles_x = (C + kTile - 1) / kTile;
    const int i0 = (blockIdx.x / tiles_x) * kTile, j0 = (blockIdx.x % tiles_x) * kTile;
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // the tile of x and g (with its +1 row and column) is loaded while the state
    // is derived
    constexpr int TE = (kTile + 1) * (kTile + 1);
    static_assert(TE <= kTrialBlock, "one tile element per thread");
    float pxv = 0.f, pgv = 0.f;
    {
        const int e = threadIdx.x;
        const int gi = i0 + e / (kTile + 1), gj = j0 + e % (kTile + 1);
        if (e < TE && gi < R && gj < C) {
            pxv = x[((long long)gi * C + gj) * B + s];
            pgv = g[((long long)gi * C + gj) * B + s];
        }
    }
    derive_state<kTrialBlock>(sS, st_in, pp, first, part_prev, s, nt, tot);
    const SliceState &S = sS; // read from LDS (a register copy of the struct spills)
    const bool apply = must_apply(S);
    const int ntr = (evaluate && !apply) ? trial_width(S, pp) : 0;
    if (!apply && ntr == 0) {
        publish_state(S, st_out, s, false);
        return;
    }
    if (threadIdx.x < TE) {
        tx[threadIdx.x / (kTile + 1)][threadIdx.x % (kTile + 1)] = pxv;
        tg[threadIdx.x / (kTile + 1)][threadIdx.x % (kTile + 1)] = pgv;
    }
    if (apply) { // x and g at a pixel are the tile's (no other workgroup writes them)
        __syncthreads();
        if (threadIdx.x < kTile * kTile) {
            const int li = threadIdx.x / kTile, lj = threadIdx.x % kTile;
            const int i = i0 + li, j = j0 + lj;
            if (i < R && j < C) {
                const long long e = ((long long)i * C + j) * B + s;
                x[e] = (float)((double)tx[li][lj] + S.s_acc * (-(double)tg[li][lj] * (1.0 / S.gn)));
            }
        }
        publish_state(S, st_out, s, true);
        return;
    }
    publish_state(S, st_out, s, false);
    const long long nslots = (long long)B * nt, slot = (long long)s * nt + blockIdx.x;
    const double inv_gn = 1.0 / S.gn;
    for (int t = threadIdx.x; t < ntr; t += kTrialBlock) coef[t] = S.s_acc + trial_beta(pp, S, S.ell + t);
    __syncthreads();
    double x00[4], x10[4], x01[4], v00[4], v10[4], v01[4];
    bool has[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        const int pix = lane + 64 * h;
        const int li = pix / kTile, lj = pix % kTile;
        const int i = i0 + li, j = j0 + lj;
        has[h] = (i <= R - 2) && (j <= C - 2);
        x00[h] = tx[li][lj];
        x10[h] = tx[li + 1][lj];
        x01[h] = tx[li][lj + 1];
        v00[h] = -(double)tg[li][lj] * inv_gn;
        v10[h] = -(double)tg[li + 1][lj] * inv_gn;
        v01[h] = -(double)tg[li][lj + 1] * inv_gn;
    }
    for (int t0 = wid * 4; t0 < ntr; t0 += W * 4) {
        double acc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            acc[k] = 0.0;
            if (t0 + k < ntr) {
                const double cf = coef[t0 + k];
#pragma unroll
                for (int h = 0; h < 4; ++h)
                    if (has[h])
                        acc[k] += tv_tau(x00[h] + cf * v00[h], x10[h] + cf * v10[h], x01[h] + cf * v01[h],
                                         pp.tv_eps2);
            }
        }
        wave_sum<4>(acc);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (t0 + k < ntr) part_out[(long long)(t0 + k) * nslots + slot] = acc[k];
        }
    }
}

// Closing launch of a phase: the decision of the last trial launch and, when
// the phase ends there, the accepted step added to x (the same arithmetic as
// the trial launches' own apply), each workgroup on its own part of x.  Where
// an earlier trial launch has applied the step already, the launch only
// carries the state over (workgroup 0 publishes it).  nt: workgroups per slice
// of the trial launches (their partials' layout).
__global__ __launch_bounds__(kTrialBlock) void k_trial_close(float *__restrict__ x, const float *__restrict__ g,
                                                             const SliceState *__restrict__ st_in,
                                                             SliceState *__restrict__ st_out, PertParams pp, int nt,
                                                             const double *__restrict__ part_prev)
{
    __shared__ double tot[kTrialChunk];
    __shared__ SliceState sS;
    const int s = blockIdx.y, B = pp.B;
    const bool lin = pp.obj == OBJ_LINEAR;
    derive_state<kTrialBlock>(sS, st_in, pp, 0, part_prev, s, nt, tot);
    const SliceState &S = sS;
    const bool apply = must_apply(S);
    if (apply) {
        const double inv_gn = 1.0 / S.gn;
        for (long long j = (long long)blockIdx.x * kTrialBlock + threadIdx.x; j < pp.n;
             j += (long long)gridDim.x * kTrialBlock) {
            const double gj = lin ? (double)g[j] : (double)g[j * B + s];
            x[j * B + s] = (float)((double)x[j * B + s] + S.s_acc * (-gj * inv_gn));
        }
    }
    publish_state(S, st_out, s, apply);
}

// The phase of the linear objective f(x) = c^T x from its direction partials
// (sum c_j^2 and sum c_j x_j per workgroup of the launch that left them).  On
// v = -c/||c|| the objective at a trial point is known in closed form,
// f(x + t v) = f(x) - t ||c||, so no trial needs a pass over x: every
// workgroup opens the phase from the partials (the same sums in the same
// order) and runs the reduction steps' trials on those values; workgroup 0
// publishes the state.  Returns whether the accepted step s v is to be added.
template <int BS>
__device__ inline bool linear_phase(SliceState &sS, const SliceState *__restrict__ st_in, const PertParams &pp,
                                   const double *__restrict__ part, int s, int nt, double *tot,
                                   SliceState *__restrict__ st_out)
{
    derive_state<BS>(sS, st_in, pp, 1, part, s, nt, tot);
    if (threadIdx.x == 0) {
        SliceState &S = sS;
        const double f = S.f_cur; // f(x^k)
        while (S.phase) { // one trial a round: bounded by n_red acceptances or the trial cap
            const double t = S.s_acc + trial_beta(pp, S, S.ell);
            const double ft = f - t * S.gn;
            record_decision(S, pp, 1, ft <= S.f_cur ? 0 : -1, ft);
        }
    }
    __syncthreads();
    const bool apply = must_apply(sS);
    publish_state(sS, st_out, s, apply);
    return apply;
}

// The linear phase in one launch: each workgroup adds the step to its own
// part of x.
__global__ __launch_bounds__(kBlock) void k_trial_linear(float *__restrict__ x, const float *__restrict__ c,
                                                         const SliceState *__restrict__ st_in,
                                                         SliceState *__restrict__ st_out, PertParams pp,
                                                         const double *__restrict__ part_phase)
{
    __shared__ double tot[kTrialChunk];
    __shared__ SliceState sS;
    const int s = blockIdx.y, B = pp.B, nt = gridDim.x;
    if (linear_phase<kBlock>(sS, st_in, pp, part_phase, s, nt, tot, st_out)) {
        const double inv_gn = 1.0 / sS.gn, s_acc = sS.s_acc;
        for (long long j = (long long)blockIdx.x * kBlock + threadIdx.x; j < pp.n; j += (long long)gridDim.x * kBlock)
            x[j * B + s] = linear_step_point(x[j * B + s], c[j], s_acc, inv_gn);
    }
}

// Trial launch for the squared norm and the linear objective (flat vectors).
__global__ __launch_bounds__(kBlock) void k_trial_flat(float *__restrict__ x, const float *__restrict__ g,
                                                       const SliceState *__restrict__ st_in,
                                                       SliceState *__restrict__ st_out, PertParams pp, int first,
                                                       int evaluate, const double *__restrict__ part_prev,
                                                       double *__restrict__ part_out)
{
    __shared__ double coef[1024];
    __shared__ double lds[4 * kTrialChunk];
    __shared__ double tot[kTrialChunk];
    __shared__ SliceState sS;
    const int s = blockIdx.y, B = pp.B, nt = gridDim.x;
    const bool lin = pp.obj == OBJ_LINEAR;
    derive_state<kBlock>(sS, st_in, pp, first, part_prev, s, nt, tot);
    const SliceState &S = sS; // read from LDS (a register copy of the struct spills)
    if (must_apply(S)) {
        const double inv_gn = 1.0 / S.gn;
        for (long long j = (long long)blockIdx.x * kBlock + threadIdx.x; j < pp.n; j += (long long)gridDim.x * kBlock) {
            const double gj = lin ? (double)g[j] : (double)g[j * B + s];
            x[j * B + s] = (float)((double)x[j * B + s] + S.s_acc * (-gj * inv_gn));
        }
        publish_state(S, st_out, s, true);
        return;
    }
    publish_state(S, st_out, s, false);
    const int ntr = evaluate ? trial_width(S, pp) : 0;
    if (ntr == 0) return;
    const long long nslots = (long long)B * nt, slot = (long long)s * nt + blockIdx.x;
    const double inv_gn = 1.0 / S.gn;
    for (int t = threadIdx.x; t < ntr; t += kBlock) coef[t] = S.s_acc + trial_beta(pp, S, S.ell + t);
    __syncthreads();
    for (int t0 = 0; t0 < ntr; t0 += kTrialChunk) {
        double acc[kTrialChunk];
#pragma unroll
        for (int w = 0; w < kTrialChunk; ++w) acc[w] = 0.0;
        for (long long j = (long long)blockIdx.x * kBlock + threadIdx.x; j < pp.n; j += (long long)gridDim.x * kBlock) {
            const double xj = (double)x[j * B + s];
            const double gj = lin ? (double)g[j] : (double)g[j * B + s];
            const double vj = -gj * inv_gn;
#pragma unroll
            for (int w = 0; w < kTrialChunk; ++w) {
                if (t0 + w < ntr) {
                    const double z = xj + coef[t0 + w] * vj;
                    acc[w] += lin ? gj * z : (pp.obj == OBJ_L1 ? fabs(z) : z * z);
                }
            }
        }
        block_sum<kTrialChunk>(acc, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int w = 0; w < kTrialChunk; ++w)
                if (t0 + w < ntr) part_out[(long long)(t0 + w) * nslots + slot] = acc[w];
        }
    }
}

// The whole perturbation phase of a flat objective in one launch, for short
// vectors (n <= kSmallPhaseMaxN): one workgroup per slice copies its entries
// of x and of the direction into LDS (float32, 8n bytes), forms ||g||^2 and
// f(x^k), opens the phase, evaluates every reduction step's trials in
// batches of kSmallTrials (the first acceptable trial in order is taken, as
// in the launch-per-batch form: the batching only decides how many trials
// are evaluated speculatively), and adds the accepted step to x.  The same
// arithmetic per entry as k_phase_flat / k_trial_flat; only the order of the
// float64 sums differs.  One workgroup is a latency chain, so every thread
// issues all of its loads of x (and c) before using any.  Reads state
// st_in[s], writes st_out[s].
template <int OBJ>
__global__ __launch_bounds__(kSmallPhaseBlock) void k_phase_small(float *__restrict__ x,
                                                                  const float *__restrict__ lin_c,
                                                                  const SliceState *__restrict__ st_in,
                                                                  SliceState *__restrict__ st_out, PertParams pp)
{
    constexpr int BS = kSmallPhaseBlock, T = kSmallTrials, U = (kSmallPhaseMaxN + BS - 1) / BS;
    extern __shared__ __align__(16) unsigned char phase_lds[];
    __shared__ double lds[(BS / 64) * T];
    __shared__ double coef[T];
    __shared__ SliceState sS;
    const int s = blockIdx.y, B = pp.B, n = (int)pp.n;
    float *xs = reinterpret_cast<float *>(phase_lds);
    float *gs = xs + n;
    if (threadIdx.x == 0) sS = st_in[s];
    __syncthreads();
    double v[2] = {0.0, 0.0}; // sum g^2, f(x^k)
    if (sS.live) {
        for (int j0 = threadIdx.x; j0 < n; j0 += U * BS) {
            float xf[U], cf[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = min(j0 + u * BS, n - 1);
                xf[u] = x[(long long)j * B + s];
                if constexpr (OBJ == OBJ_LINEAR) cf[u] = lin_c[j];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = j0 + u * BS;
                if (j >= n) break;
                const double xj = (double)xf[u];
                float gf;
                if constexpr (OBJ == OBJ_SQNORM) {
                    v[1] += xj * xj;
                    gf = (float)(2.0 * xj);
                } else if constexpr (OBJ == OBJ_L1) { // subgradient sign(x), 0 at 0
                    v[1] += fabs(xj);
                    gf = xj > 0.0 ? 1.f : (xj < 0.0 ? -1.f : 0.f);
                } else {
                    gf = cf[u];
                    v[1] += (double)gf * xj;
                }
                v[0] += (double)gf * (double)gf;
                xs[j] = xf[u];
                gs[j] = gf;
            }
        }
    }
    block_sum<2, BS>(v, lds); // its barriers also publish xs and gs
    if (threadIdx.x == 0) open_phase_state(sS, pp, v[0], v[1]);
    __syncthreads();
    while (sS.phase) { // sS changes only in thread 0, between barriers
        const int ntr = min(T, pp.max_trials - sS.step_tried);
        if (threadIdx.x < ntr) coef[threadIdx.x] = sS.s_acc + trial_beta(pp, sS, sS.ell + threadIdx.x);
        __syncthreads();
        const double inv_gn = 1.0 / sS.gn;
        double acc[T], cw[T];
#pragma unroll
        for (int w = 0; w < T; ++w) {
            acc[w] = 0.0;
            cw[w] = w < ntr ? coef[w] : 0.0;
        }
#pragma unroll 4
        for (int j = threadIdx.x; j < n; j += BS) {
            const double xj = (double)xs[j], gj = (double)gs[j], vj = -gj * inv_gn;
#pragma unroll
            for (int w = 0; w < T; ++w) {
                if (w < ntr) {
                    const double z = xj + cw[w] * vj;
                    if constexpr (OBJ == OBJ_LINEAR) acc[w] += gj * z;
                    else if constexpr (OBJ == OBJ_L1) acc[w] += fabs(z);
                    else acc[w] += z * z;
                }
            }
        }
        block_sum<T, BS>(acc, lds);
        if (threadIdx.x == 0) {
            int t = -1;
            for (int w = 0; w < ntr; ++w)
                if (acc[w] <= sS.f_cur) {
                    t = w;
                    break;
                }
            record_decision(sS, pp, ntr, t, t >= 0 ? acc[t] : 0.0);
        }
        __syncthreads();
    }
    const bool apply = must_apply(sS);
    if (apply) {
        const double inv_gn = 1.0 / sS.gn;
#pragma unroll 4
        for (int j = threadIdx.x; j < n; j += BS)
            x[(long long)j * B + s] = (float)((double)xs[j] + sS.s_acc * (-(double)gs[j] * inv_gn));
    }
    if (threadIdx.x == 0) {
        SliceState o = sS;
        if (apply) o.applied = 1;
        st_out[s] = o;
    }
}

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------

template <typename VT>
__device__ inline float stored_value(const void *val, long long p);
template <>
__device__ inline float stored_value<float>(const void *val, long long p) { return static_cast<const float *>(val)[p]; }
template <>
__device__ inline float stored_value<Bf16Tag>(const void *val, long long p)
{
    return __uint_as_float((uint32_t) static_cast<const uint16_t *>(val)[p] << 16);
}
template <>
__device__ inline float stored_value<F16Tag>(const void *val, long long p)
{
    return __half2float(__ushort_as_half(static_cast<const uint16_t *>(val)[p]));
}
template <>
__device__ inline float stored_value<Bf16PTag>(const void *val, long long p)
{
    return bf16_lo(static_cast<const uint32_t *>(val)[p]);
}
template <>
__device__ inline float stored_value<F16PTag>(const void *val, long long p)
{
    return f16_lo(static_cast<const uint32_t *>(val)[p]);
}

// q_i = ||a_i||^2 in float64 from the stored (possibly rounded) values; one wave per row
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_rownorm(SpView A, double *__restrict__ q)
{
    const int lane = threadIdx.x & 63;
    const long long row = (long long)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (row >= A.rows) return;
    const int beg = A.ptr[row], end = A.ptr[row + 1];
    double s = 0.0;
    for (int p = beg + lane; p < end; p += 64) {
        const double a = (double)stored_value<VT>(A.val, p) * (double)A.vscale_inv;
        s += a * a;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) q[row] = s;
}

__global__ void k_make_D(const double *__restrict__ q, const double *__restrict__ w, float *__restrict__ D, long long m)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (long long)gridDim.x * blockDim.x)
        D[i] = q[i] > 0.0 ? (float)(w[i] / q[i]) : 0.f;
}

__global__ void k_to_bf16(const float *__restrict__ src, uint16_t *__restrict__ dst, long long count)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
        dst[i] = __bfloat16_as_ushort(__float2bfloat16(src[i]));
}

__global__ void k_to_f16(const float *__restrict__ src, uint16_t *__restrict__ dst, long long count, float scale)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
        dst[i] = __half_as_ushort(__float2half_rn(src[i] * scale));
}

__global__ void k_pack16u(const uint16_t *__restrict__ val16, const uint16_t *__restrict__ idx16,
                          uint32_t *__restrict__ packed, long long count)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
        packed[i] = (uint32_t)val16[i] | ((uint32_t)idx16[i] << 16);
}

__global__ void k_pack16(const uint16_t *__restrict__ val16, const int32_t *__restrict__ idx,
                         uint32_t *__restrict__ packed, long long count)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
        packed[i] = (uint32_t)val16[i] | ((uint32_t)idx[i] << 16);
}

__global__ void k_fill(float *__restrict__ p, float v, long long count)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_init_state(SliceState *st, int B, StopParams sp)
{
    const int s = threadIdx.x;
    if (s >= B) return;
    SliceState S;
    S.f_cur = S.f_start = __longlong_as_double(0x7ff8000000000000LL);
    S.gn = 0.0;
    S.s_acc = 0.0;
    S.prox = __longlong_as_double(0x7ff8000000000000LL);
    S.k = 0;
    S.k_end = 0x7fffffffffffffffLL;
    S.ell = 0;
    S.restarts = 0;
    S.trials = S.accepts = S.cap_hits = 0;
    S.n_done = 0;
    S.phase = 0;
    S.step_tried = 0;
    S.trials_it = S.accepts_it = 0;
    S.live = 1;
    S.applied = 0;
    S.enabled = 1;
    S.nonfinite = 0;
    S.need_last = 0;
    S.stop_on = sp.on;
    S.stop_n = sp.n;
    S.stop_max = sp.max_iters;
    S.stop_prox = sp.prox;
    S.stop_dprox = sp.dprox;
    S.stop_dobj = sp.dobj;
    S.stop_var = sp.var;
    S.stop_reason = STOP_NONE;
    S.dp_run = S.feas_ok = S.ran = 0;
    S.p_last = S.f_last = S.f_ref = __longlong_as_double(0x7ff8000000000000LL);
    S.beta_ad = 0.0;
    S.var_n = S.var_mean = S.var_m2 = 0.0;
    st[s] = S;
}

// Column s of a slice-interleaved [rows x B] array, in or out.
__global__ void k_put_column(float *__restrict__ dst, const float *__restrict__ src, long long rows, int B, int s)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += (long long)gridDim.x * blockDim.x)
        dst[i * B + s] = src[i];
}

// Validation of a slot's bands staged on the device.  flag[0] collects bit 0
// for a NaN bound and bit 1 for lower > upper, flag[1] the lowest row with
// either; k_slot_flag_clear sets them to {0, 0xffffffff} first.
__global__ void k_slot_flag_clear(unsigned *flag)
{
    if (threadIdx.x == 0) {
        flag[0] = 0u;
        flag[1] = 0xffffffffu;
    }
}

__global__ void k_check_bands(const float *__restrict__ lo, const float *__restrict__ up, long long m,
                              unsigned *__restrict__ flag)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (long long)gridDim.x * blockDim.x) {
        const float a = lo[i], b = up[i];
        const unsigned bits = (isnan(a) || isnan(b)) ? 1u : (a > b ? 2u : 0u);
        if (bits) {
            atomicOr(&flag[0], bits);
            atomicMin(&flag[1], (unsigned)i);
        }
    }
}

__global__ void k_get_column(float *__restrict__ dst, const float *__restrict__ src, long long rows, int B, int s)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += (long long)gridDim.x * blockDim.x)
        dst[i] = src[i * B + s];
}

// Slot s starts afresh: k = ell = restarts = 0, counters 0, `budget`
// iterations to run (0 disables the slot).
__global__ void k_reset_slot(SliceState *st, int s, long long budget)
{
    if (threadIdx.x != 0) return;
    SliceState S = st[s];
    S.f_cur = S.f_start = __longlong_as_double(0x7ff8000000000000LL);
    S.gn = 0.0;
    S.s_acc = 0.0;
    S.prox = __longlong_as_double(0x7ff8000000000000LL);
    S.k = 0;
    S.k_end = budget;
    S.ell = 0;
    S.restarts = 0;
    S.trials = S.accepts = S.cap_hits = 0;
    S.n_done = 0;
    S.phase = 0;
    S.step_tried = 0;
    S.trials_it = S.accepts_it = 0;
    S.enabled = budget > 0 ? 1 : 0;
    S.live = S.enabled;
    S.applied = 0;
    S.nonfinite = 0;
    S.need_last = 0;
    S.stop_reason = STOP_NONE;
    S.dp_run = S.feas_ok = S.ran = 0;
    S.p_last = S.f_last = S.f_ref = __longlong_as_double(0x7ff8000000000000LL);
    S.beta_ad = 0.0;
    S.var_n = S.var_mean = S.var_m2 = 0.0;
    st[s] = S;
}

__global__ void k_disable_slot(SliceState *st, int s)
{
    if (threadIdx.x != 0) return;
    st[s].enabled = 0;
    st[s].live = 0;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline unsigned grid_for(long long work, int per_block, unsigned cap)
{
    long long g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

hipError_t launch_rownorm(const SpView &A, int vk, double *q, hipStream_t s)
{
    const unsigned grid = grid_for(A.rows, kBlock / 64, 1u << 30);
    switch (vk) {
    case VK_F32: hipLaunchKernelGGL(k_rownorm<float>, dim3(grid), dim3(kBlock), 0, s, A, q); break;
    case VK_BF16: hipLaunchKernelGGL(k_rownorm<Bf16Tag>, dim3(grid), dim3(kBlock), 0, s, A, q); break;
    case VK_F16: hipLaunchKernelGGL(k_rownorm<F16Tag>, dim3(grid), dim3(kBlock), 0, s, A, q); break;
    case VK_BF16P: hipLaunchKernelGGL(k_rownorm<Bf16PTag>, dim3(grid), dim3(kBlock), 0, s, A, q); break;
    case VK_F16P: hipLaunchKernelGGL(k_rownorm<F16PTag>, dim3(grid), dim3(kBlock), 0, s, A, q); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_make_D(const double *q, const double *w, float *D, int64_t m, hipStream_t s)
{
    hipLaunchKernelGGL(k_make_D, dim3(grid_for(m, kBlock, 4096)), dim3(kBlock), 0, s, q, w, D, (long long)m);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *src, uint16_t *dst, int64_t count, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(count, kBlock, 8192)), dim3(kBlock), 0, s, src, dst, (long long)count);
    return hipGetLastError();
}

hipError_t launch_to_f16(const float *src, uint16_t *dst, int64_t count, float scale, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_f16, dim3(grid_for(count, kBlock, 8192)), dim3(kBlock), 0, s, src, dst, (long long)count,
                       scale);
    return hipGetLastError();
}

hipError_t launch_pack16u(const uint16_t *val16, const uint16_t *idx16, uint32_t *packed, int64_t count, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack16u, dim3(grid_for(count, kBlock, 8192)), dim3(kBlock), 0, s, val16, idx16, packed,
                       (long long)count);
    return hipGetLastError();
}

hipError_t launch_pack16(const uint16_t *val16, const int32_t *idx, uint32_t *packed, int64_t count, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack16, dim3(grid_for(count, kBlock, 8192)), dim3(kBlock), 0, s, val16, idx, packed,
                       (long long)count);
    return hipGetLastError();
}

hipError_t launch_fill(float *p, float v, int64_t count, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3(grid_for(count, kBlock, 4096)), dim3(kBlock), 0, s, p, v, (long long)count);
    return hipGetLastError();
}

hipError_t launch_put_column(float *dst, const float *src, int64_t rows, int B, int slot, hipStream_t s)
{
    hipLaunchKernelGGL(k_put_column, dim3(grid_for(rows, kBlock, 2048)), dim3(kBlock), 0, s, dst, src, (long long)rows, B,
                       slot);
    return hipGetLastError();
}

hipError_t launch_check_bands(const float *lo, const float *up, int64_t m, unsigned *flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_slot_flag_clear, dim3(1), dim3(64), 0, s, flag);
    hipLaunchKernelGGL(k_check_bands, dim3(grid_for(m, kBlock, 2048)), dim3(kBlock), 0, s, lo, up, (long long)m, flag);
    return hipGetLastError();
}

hipError_t launch_get_column(float *dst, const float *src, int64_t rows, int B, int slot, hipStream_t s)
{
    hipLaunchKernelGGL(k_get_column, dim3(grid_for(rows, kBlock, 2048)), dim3(kBlock), 0, s, dst, src, (long long)rows, B,
                       slot);
    return hipGetLastError();
}

hipError_t launch_reset_slot(SliceState *st, int slot, int64_t budget, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset_slot, dim3(1), dim3(64), 0, s, st, slot, (long long)budget);
    return hipGetLastError();
}

hipError_t launch_disable_slot(SliceState *st, int slot, hipStream_t s)
{
    hipLaunchKernelGGL(k_disable_slot, dim3(1), dim3(64), 0, s, st, slot);
    return hipGetLastError();
}

hipError_t launch_init_state(SliceState *st, int B, StopParams sp, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, s, st, B, sp);
    return hipGetLastError();
}

template <typename VT, int VEC>
static hipError_t pass1_vec(const PassCfg &cfg, const SpView &A, const float *x, const float *lower,
                            const float *upper, RowW w, float *c, const SliceState *st, int query,
                            double *partials, hipStream_t s)
{
    const dim3 grid(cfg.grid), block(kBlock);
    if constexpr (VEC == 1) { // interleaved lanes: 8 to 64 lanes per row
        switch (cfg.lpr) {
        case 8: hipLaunchKernelGGL((k_pass1<8, 1, VT>), grid, block, 0, s, A, x, lower, upper, w, c, st, query, partials); break;
        case 16: hipLaunchKernelGGL((k_pass1<16, 1, VT>), grid, block, 0, s, A, x, lower, upper, w, c, st, query, partials); break;
        case 32: hipLaunchKernelGGL((k_pass1<32, 1, VT>), grid, block, 0, s, A, x, lower, upper, w, c, st, query, partials); break;
        case 64: hipLaunchKernelGGL((k_pass1<64, 1, VT>), grid, block, 0, s, A, x, lower, upper, w, c, st, query, partials); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (cfg.lpr) {
    case 2: hipLaunchKernelGGL((k_pass1<2, VEC, VT>), grid, block, 0, s, A, x, lower, upper, w, c, st, query, partials); break;
    case 4: hipLaunchKernelGGL((k_pass1<4, VEC, VT>), grid, block, 0, s, A, x, lower, upper, w, c, st, query, partials); break;
    case 8: hipLaunchKernelGGL((k_pass1<8, VEC, VT>), grid, block, 0, s, A, x, lower, upper, w, c, st, query, partials); break;
    case 16: hipLaunchKernelGGL((k_pass1<16, VEC, VT>), grid, block, 0, s, A, x, lower, upper, w, c, st, query, partials); break;
    case 32: hipLaunchKernelGGL((k_pass1<32, VEC, VT>), grid, block, 0, s, A, x, lower, upper, w, c, st, query, partials); break;
    case 64: hipLaunchKernelGGL((k_pass1<64, VEC, VT>), grid, block, 0, s, A, x, lower, upper, w, c, st, query, partials); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename VT, int VEC>
static hipError_t pass1_stream(const PassCfg &cfg, const SpView &A, const RowBlocks &RB, const float *x,
                               const float *lower, const float *upper, RowW w, float *c,
                               const SliceState *st, int query, double *partials, hipStream_t s)
{
    hipLaunchKernelGGL((k_pass1_stream<VEC, VT>), dim3(cfg.grid), dim3(kBlock), 0, s, A, RB, x, lower, upper, w, c,
                       st, query, partials);
    return hipGetLastError();
}

template <typename VT, int VEC, int B>
static hipError_t pass1_mm(const PassCfg &cfg, const SpView &A, const float *x, const float *lower,
                           const float *upper, RowW w, float *c, const SliceState *st, int query,
                           double *partials, hipStream_t s)
{
    const dim3 grid(cfg.grid), block(kBlock);
    switch (cfg.lpr) {
    case 4: hipLaunchKernelGGL((k_pass1_mm<4, VEC, VT, B>), grid, block, 0, s, A, x, lower, upper, w, c, st, query, partials); break;
    case 8: hipLaunchKernelGGL((k_pass1_mm<8, VEC, VT, B>), grid, block, 0, s, A, x, lower, upper, w, c, st, query, partials); break;
    case 16: hipLaunchKernelGGL((k_pass1_mm<16, VEC, VT, B>), grid, block, 0, s, A, x, lower, upper, w, c, st, query, partials); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename VT, int VEC>
static hipError_t pass1_mm_b(const PassCfg &cfg, const SpView &A, const float *x, const float *lower,
                             const float *upper, RowW w, float *c, const SliceState *st, int B, int query,
                             double *partials, hipStream_t s)
{
    switch (B) {
    case 2: return pass1_mm<VT, VEC, 2>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
    case 4: return pass1_mm<VT, VEC, 4>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
    case 8: return pass1_mm<VT, VEC, 8>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
    case 16: return pass1_mm<VT, VEC, 16>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
    case 32: return pass1_mm<VT, VEC, 32>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename VT, int VEC, int LPR>
static hipError_t pass1_lds_go(const PassCfg &cfg, const SpView &A, const float *x, const float *lower,
                               const float *upper, RowW w, float *c, const SliceState *st, int query,
                               double *partials, int prepare, hipStream_t s)
{
    auto kern = k_pass1_lds<LPR, VEC, VT>;
    if (prepare)
        return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)(sizeof(float) * kLdsPassFloats));
    const size_t shm = sizeof(float4) * size_t((cfg.xlds + 3) / 4);
    hipLaunchKernelGGL(kern, dim3(cfg.grid), dim3(kLdsPassBlock), shm, s, A, x, cfg.xlds, lower, upper, w, c, st,
                       query, partials);
    return hipGetLastError();
}

template <typename VT, int VEC>
static hipError_t pass1_lds(const PassCfg &cfg, const SpView &A, const float *x, const float *lower,
                            const float *upper, RowW w, float *c, const SliceState *st, int query, double *partials,
                            int prepare, hipStream_t s)
{
    switch (cfg.lpr) {
    case 4: return pass1_lds_go<VT, VEC, 4>(cfg, A, x, lower, upper, w, c, st, query, partials, prepare, s);
    case 8: return pass1_lds_go<VT, VEC, 8>(cfg, A, x, lower, upper, w, c, st, query, partials, prepare, s);
    case 16: return pass1_lds_go<VT, VEC, 16>(cfg, A, x, lower, upper, w, c, st, query, partials, prepare, s);
    case 32: return pass1_lds_go<VT, VEC, 32>(cfg, A, x, lower, upper, w, c, st, query, partials, prepare, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename VT>
static hipError_t pass1_lds_v(const PassCfg &cfg, const SpView &A, const float *x, const float *lower,
                              const float *upper, RowW w, float *c, const SliceState *st, int query, double *partials,
                              int prepare, hipStream_t s)
{
    if (cfg.vec == 8) return pass1_lds<VT, 8>(cfg, A, x, lower, upper, w, c, st, query, partials, prepare, s);
    if (cfg.vec == 4) return pass1_lds<VT, 4>(cfg, A, x, lower, upper, w, c, st, query, partials, prepare, s);
    return hipErrorInvalidValue;
}

static hipError_t pass1_lds_kind(const PassCfg &cfg, int vk, const SpView &A, const float *x, const float *lower,
                                 const float *upper, RowW w, float *c, const SliceState *st, int query,
                                 double *partials, int prepare, hipStream_t s)
{
    switch (vk) {
    case VK_F32U16: return pass1_lds_v<F32U16Tag>(cfg, A, x, lower, upper, w, c, st, query, partials, prepare, s);
    case VK_F32: return pass1_lds_v<float>(cfg, A, x, lower, upper, w, c, st, query, partials, prepare, s);
    case VK_BF16: return pass1_lds_v<Bf16Tag>(cfg, A, x, lower, upper, w, c, st, query, partials, prepare, s);
    case VK_BF16P: return pass1_lds_v<Bf16PTag>(cfg, A, x, lower, upper, w, c, st, query, partials, prepare, s);
    case VK_F16: return pass1_lds_v<F16Tag>(cfg, A, x, lower, upper, w, c, st, query, partials, prepare, s);
    case VK_F16P: return pass1_lds_v<F16PTag>(cfg, A, x, lower, upper, w, c, st, query, partials, prepare, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename VT, int VEC, int LPR>
static hipError_t pass2_lds_go(const PassCfg &cfg, const SpView &At, const float *c, float *x, ColStep cs,
                               const SliceState *st_in, SliceState *st_out, const double *part1, int nparts1, Hist h,
                               int prepare, hipStream_t s)
{
    auto kern = k_pass2_lds<LPR, VEC, VT>;
    if (prepare)
        return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)(sizeof(float) * kLdsPassFloats));
    const size_t shm = sizeof(float4) * size_t((cfg.xlds + 3) / 4);
    hipLaunchKernelGGL(kern, dim3(cfg.grid), dim3(kLdsPassBlock), shm, s, At, c, cfg.xlds, x, cs, st_in, st_out,
                       part1, nparts1, h);
    return hipGetLastError();
}

template <typename VT, int VEC>
static hipError_t pass2_lds(const PassCfg &cfg, const SpView &At, const float *c, float *x, ColStep cs,
                            const SliceState *st_in, SliceState *st_out, const double *part1, int nparts1, Hist h,
                            int prepare, hipStream_t s)
{
    switch (cfg.lpr) {
    case 4: return pass2_lds_go<VT, VEC, 4>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, prepare, s);
    case 8: return pass2_lds_go<VT, VEC, 8>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, prepare, s);
    case 16: return pass2_lds_go<VT, VEC, 16>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, prepare, s);
    case 32: return pass2_lds_go<VT, VEC, 32>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, prepare, s);
    default: return hipErrorInvalidValue;
    }
}

static hipError_t pass2_lds_kind(const PassCfg &cfg, int vk, const SpView &At, const float *c, float *x, ColStep cs,
                                 const SliceState *st_in, SliceState *st_out, const double *part1, int nparts1, Hist h,
                                 int prepare, hipStream_t s)
{
#define SMX_P2L(VT)                                                                                                    \
    (cfg.vec == 8 ? pass2_lds<VT, 8>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, prepare, s)                 \
                  : (cfg.vec == 4 ? pass2_lds<VT, 4>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, prepare, s) \
                                  : hipErrorInvalidValue))
    switch (vk) {
    case VK_F32U16: return SMX_P2L(F32U16Tag);
    case VK_F32: return SMX_P2L(float);
    case VK_BF16: return SMX_P2L(Bf16Tag);
    case VK_BF16P: return SMX_P2L(Bf16PTag);
    case VK_F16: return SMX_P2L(F16Tag);
    case VK_F16P: return SMX_P2L(F16PTag);
    default: return hipErrorInvalidValue;
    }
#undef SMX_P2L
}

template <typename VT, int VEC, int LPR>
static hipError_t panel_go(const PassCfg &cfg, const SpView &At, const PanelView &PV, const float *c,
                           const SliceState *st_in, int prepare, hipStream_t s)
{
    auto kern = k_pass2_panel<LPR, VEC, VT>;
    if (prepare)
        return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)(sizeof(float) * kLdsPassFloats));
    const int n = (int)At.rows;
    const int chunks = std::max(1, std::min(n, (4 * cfg.grid + PV.np - 1) / PV.np)); // ~4 work items per workgroup
    const int cpt = (n + chunks - 1) / chunks;
    const size_t shm = sizeof(float4) * size_t((PV.P + 3) / 4);
    hipLaunchKernelGGL(kern, dim3(cfg.grid), dim3(kLdsPassBlock), shm, s, At, PV.pp, PV.np, PV.P, PV.m, cpt,
                       (n + cpt - 1) / cpt, PV.local, c, PV.ypanel, st_in);
    return hipGetLastError();
}

template <typename VT, int VEC>
static hipError_t panel_lpr(const PassCfg &cfg, const SpView &At, const PanelView &PV, const float *c,
                            const SliceState *st_in, int prepare, hipStream_t s)
{
    switch (cfg.lpr) {
    case 8: return panel_go<VT, VEC, 8>(cfg, At, PV, c, st_in, prepare, s);
    case 16: return panel_go<VT, VEC, 16>(cfg, At, PV, c, st_in, prepare, s);
    case 32: return panel_go<VT, VEC, 32>(cfg, At, PV, c, st_in, prepare, s);
    case 64: return panel_go<VT, VEC, 64>(cfg, At, PV, c, st_in, prepare, s);
    default: return hipErrorInvalidValue;
    }
}

static hipError_t panel_kind(const PassCfg &cfg, int vk, const SpView &At, const PanelView &PV, const float *c,
                             const SliceState *st_in, int prepare, hipStream_t s)
{
#define SMX_PAN(VT)                                                                                                    \
    (cfg.vec == 8 ? panel_lpr<VT, 8>(cfg, At, PV, c, st_in, prepare, s)                                              \
                  : (cfg.vec == 4 ? panel_lpr<VT, 4>(cfg, At, PV, c, st_in, prepare, s) : hipErrorInvalidValue))
    switch (vk) {
    case VK_F32U16: return SMX_PAN(F32U16Tag);
    case VK_F32: return SMX_PAN(float);
    case VK_BF16: return SMX_PAN(Bf16Tag);
    case VK_BF16P: return SMX_PAN(Bf16PTag);
    case VK_F16: return SMX_PAN(F16Tag);
    case VK_F16P: return SMX_PAN(F16PTag);
    default: return hipErrorInvalidValue;
    }
#undef SMX_PAN
}

hipError_t launch_pass2_panels(const PassCfg &cfg, const SpView &At, const PanelView &PV, int vk, const float *c,
                               float *x, ColStep cs, const SliceState *st_in, SliceState *st_out, const double *part1,
                               int nparts1, Hist h, hipStream_t s)
{
    if (cfg.grid < 1 || cfg.grid > kMaxPassGrid || nparts1 < 1 || nparts1 > kMaxPassGrid) return hipErrorInvalidValue;
    if (PV.np < 1 || PV.P < 1 || PV.P > kLdsPassFloats || PV.P % 4 != 0 || PV.m < 1 ||
        (long long)PV.np * PV.P < PV.m || (long long)(PV.np - 1) * PV.P >= PV.m || !PV.pp || !PV.ypanel)
        return hipErrorInvalidValue;
    const hipError_t e = panel_kind(cfg, vk, At, PV, c, st_in, 0, s);
    if (e != hipSuccess) return e;
    // the column sums in the same grid, so that the ||y||^2 partials of the
    // extrapolated steps number cfg.grid as for the other pass-2 shapes
    hipLaunchKernelGGL(k_pass2_panel_sum, dim3(cfg.grid), dim3(kBlock), 0, s, PV.np, (int)At.rows, PV.ypanel,
                       At.vscale_inv, x, cs, st_in, st_out, part1, nparts1, h);
    return hipGetLastError();
}

hipError_t prepare_lds_passes()
{
    static hipError_t done = hipErrorNotReady;
    if (done == hipSuccess) return done;
    const SpView none{};
    for (int vk : {VK_F32U16, VK_F32, VK_BF16, VK_BF16P, VK_F16, VK_F16P})
        for (int lpr : {4, 8, 16, 32})
            for (int vec : {4, 8}) {
                PassCfg c;
                c.mode = 3;
                c.lpr = lpr;
                c.vec = vec;
                c.grid = 1;
                hipError_t e = pass1_lds_kind(c, vk, none, nullptr, nullptr, nullptr, RowW{}, nullptr, nullptr, 0,
                                              nullptr, 1, nullptr);
                if (e != hipSuccess) return e;
                e = pass2_lds_kind(c, vk, none, nullptr, nullptr, ColStep{}, nullptr, nullptr, nullptr, 0, Hist{}, 1,
                                   nullptr);
                if (e != hipSuccess) return e;
                for (int plpr : {8, 16, 32, 64}) {
                    PassCfg cp = c;
                    cp.lpr = plpr;
                    e = panel_kind(cp, vk, none, PanelView{}, nullptr, nullptr, 1, nullptr);
                    if (e != hipSuccess) return e;
                }
            }
    done = hipSuccess;
    return done;
}

hipError_t launch_pass1(const PassCfg &cfg, const SpView &A, const RowBlocks &RB, int vk, const float *x,
                        const float *lower, const float *upper, RowW w, float *c, const SliceState *st, int B,
                        int query, double *partials, hipStream_t s)
{
    if (cfg.grid < 1 || cfg.grid > kMaxPassGrid) return hipErrorInvalidValue;
    if (cfg.mode == 3) {
        if (B != 1 || cfg.xlds < 1 || cfg.xlds > kLdsPassFloats) return hipErrorInvalidValue;
        return pass1_lds_kind(cfg, vk, A, x, lower, upper, w, c, st, query, partials, 0, s);
    }
    if (B > 1) {
        if (vk == VK_F32U16) return hipErrorInvalidValue;
        if (vk == VK_F32) return pass1_mm_b<float, 4>(cfg, A, x, lower, upper, w, c, st, B, query, partials, s);
        if (vk == VK_BF16) return pass1_mm_b<Bf16Tag, 8>(cfg, A, x, lower, upper, w, c, st, B, query, partials, s);
        if (vk == VK_BF16P) return pass1_mm_b<Bf16PTag, 4>(cfg, A, x, lower, upper, w, c, st, B, query, partials, s);
        if (vk == VK_F16P) return pass1_mm_b<F16PTag, 4>(cfg, A, x, lower, upper, w, c, st, B, query, partials, s);
        return pass1_mm_b<F16Tag, 8>(cfg, A, x, lower, upper, w, c, st, B, query, partials, s);
    }
    if (cfg.mode == 1) {
        if (vk == VK_F32U16) return pass1_stream<F32U16Tag, 4>(cfg, A, RB, x, lower, upper, w, c, st, query, partials, s);
        if (vk == VK_F32) return pass1_stream<float, 4>(cfg, A, RB, x, lower, upper, w, c, st, query, partials, s);
        if (vk == VK_BF16) return pass1_stream<Bf16Tag, 8>(cfg, A, RB, x, lower, upper, w, c, st, query, partials, s);
        if (vk == VK_BF16P) return pass1_stream<Bf16PTag, 4>(cfg, A, RB, x, lower, upper, w, c, st, query, partials, s);
        if (vk == VK_F16P) return pass1_stream<F16PTag, 4>(cfg, A, RB, x, lower, upper, w, c, st, query, partials, s);
        return pass1_stream<F16Tag, 8>(cfg, A, RB, x, lower, upper, w, c, st, query, partials, s);
    }
    if (vk == VK_BF16P) {
        if (cfg.vec == 1) return pass1_vec<Bf16PTag, 1>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
        if (cfg.vec == 8) return pass1_vec<Bf16PTag, 8>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
        return pass1_vec<Bf16PTag, 4>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
    }
    if (vk == VK_F16P) {
        if (cfg.vec == 1) return pass1_vec<F16PTag, 1>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
        if (cfg.vec == 8) return pass1_vec<F16PTag, 8>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
        return pass1_vec<F16PTag, 4>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
    }
    if (vk == VK_F32U16) {
        if (cfg.vec == 1) return pass1_vec<F32U16Tag, 1>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
        if (cfg.vec == 8) return pass1_vec<F32U16Tag, 8>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
        return pass1_vec<F32U16Tag, 4>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
    }
    if (vk == VK_F32) {
        if (cfg.vec == 1) return pass1_vec<float, 1>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
        if (cfg.vec == 8) return pass1_vec<float, 8>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
        return pass1_vec<float, 4>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
    }
    if (vk == VK_BF16) {
        if (cfg.vec == 1) return pass1_vec<Bf16Tag, 1>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
        if (cfg.vec == 8) return pass1_vec<Bf16Tag, 8>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
        return pass1_vec<Bf16Tag, 4>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
    }
    if (cfg.vec == 1) return pass1_vec<F16Tag, 1>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
    if (cfg.vec == 8) return pass1_vec<F16Tag, 8>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
    return pass1_vec<F16Tag, 4>(cfg, A, x, lower, upper, w, c, st, query, partials, s);
}

template <typename VT, int VEC>
static hipError_t pass2_vec(const PassCfg &cfg, const SpView &At, const float *c, float *x, ColStep cs,
                            const SliceState *st_in, SliceState *st_out, const double *part1, int nparts1, Hist h,
                            hipStream_t s)
{
    const dim3 grid(cfg.grid), block(kBlock);
#define SMX_P2(L) hipLaunchKernelGGL((k_pass2<L, VEC, VT>), grid, block, 0, s, At, c, x, cs, st_in, st_out, part1, nparts1, h)
    switch (cfg.lpr) {
    case 2: SMX_P2(2); break;
    case 4: SMX_P2(4); break;
    case 8: SMX_P2(8); break;
    case 16: SMX_P2(16); break;
    case 32: SMX_P2(32); break;
    case 64: SMX_P2(64); break;
    default: return hipErrorInvalidValue;
    }
#undef SMX_P2
    return hipGetLastError();
}

template <typename VT, int VEC>
static hipError_t pass2_stream(const PassCfg &cfg, const SpView &At, const RowBlocks &RB, const float *c, float *x,
                               ColStep cs, const SliceState *st_in, SliceState *st_out, const double *part1,
                               int nparts1, Hist h, hipStream_t s)
{
    hipLaunchKernelGGL((k_pass2_stream<VEC, VT>), dim3(cfg.grid), dim3(kBlock), 0, s, At, RB, c, x, cs,
                       st_in, st_out, part1, nparts1, h);
    return hipGetLastError();
}

template <typename VT, int VEC, int B>
static hipError_t pass2_mm(const PassCfg &cfg, const SpView &At, const float *c, float *x, ColStep cs,
                           const SliceState *st_in, SliceState *st_out, const double *part1, int nparts1, Hist h,
                           hipStream_t s)
{
    const dim3 grid(cfg.grid), block(kBlock);
#define SMX_P2MM(L) hipLaunchKernelGGL((k_pass2_mm<L, VEC, VT, B>), grid, block, 0, s, At, c, x, cs, st_in, st_out, part1, nparts1, h)
    switch (cfg.lpr) {
    case 4: SMX_P2MM(4); break;
    case 8: SMX_P2MM(8); break;
    case 16: SMX_P2MM(16); break;
    default: return hipErrorInvalidValue;
    }
#undef SMX_P2MM
    return hipGetLastError();
}

template <typename VT, int VEC>
static hipError_t pass2_mm_b(const PassCfg &cfg, const SpView &At, const float *c, float *x, ColStep cs,
                             const SliceState *st_in, SliceState *st_out, int B, const double *part1, int nparts1,
                             Hist h, hipStream_t s)
{
    switch (B) {
    case 2: return pass2_mm<VT, VEC, 2>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    case 4: return pass2_mm<VT, VEC, 4>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    case 8: return pass2_mm<VT, VEC, 8>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    case 16: return pass2_mm<VT, VEC, 16>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    case 32: return pass2_mm<VT, VEC, 32>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename VT, int VEC, int B>
static hipError_t pass2_tiles_mm(const PassCfg &cfg, const TileView &T, const float *c, float *x, ColStep cs,
                                 const SliceState *st_in, SliceState *st_out, const double *part1, int nparts1,
                                 Hist h, hipStream_t s)
{
    const dim3 grid(cfg.grid), block(kBlock);
    const size_t shm = sizeof(float) * B * size_t(T.max_rows > 0 ? T.max_rows : 1);
#define SMX_P2TM(L) hipLaunchKernelGGL((k_pass2_tile_mm<L, VEC, VT, B>), grid, block, shm, s, T, c, x, cs, st_in, st_out, part1, nparts1, h)
    switch (cfg.lpr) {
    case 2: SMX_P2TM(2); break;
    case 4: SMX_P2TM(4); break;
    case 8: SMX_P2TM(8); break;
    case 16: SMX_P2TM(16); break;
    default: return hipErrorInvalidValue;
    }
#undef SMX_P2TM
    return hipGetLastError();
}

template <typename VT, int VEC>
static hipError_t pass2_tiles_b(const PassCfg &cfg, const TileView &T, const float *c, float *x, ColStep cs,
                                const SliceState *st_in, SliceState *st_out, int B, const double *part1,
                                int nparts1, Hist h, hipStream_t s)
{
    switch (B) {
    case 2: return pass2_tiles_mm<VT, VEC, 2>(cfg, T, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    case 4: return pass2_tiles_mm<VT, VEC, 4>(cfg, T, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    case 8: return pass2_tiles_mm<VT, VEC, 8>(cfg, T, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    case 16: return pass2_tiles_mm<VT, VEC, 16>(cfg, T, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    case 32: return pass2_tiles_mm<VT, VEC, 32>(cfg, T, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename VT, int VEC>
hipError_t pass2_tiles(const PassCfg &cfg, const TileView &T, const float *c, float *x, ColStep cs,
                       const SliceState *st_in, SliceState *st_out, const double *part1, int nparts1, Hist h,
                       hipStream_t s)
{
    const dim3 grid(cfg.grid), block(kBlock);
    const size_t shm = sizeof(float) * size_t(T.max_rows > 0 ? T.max_rows : 1);
#define SMX_P2T(L) hipLaunchKernelGGL((k_pass2_tile<L, VEC, VT>), grid, block, shm, s, T, c, x, cs, st_in, st_out, part1, nparts1, h)
    switch (cfg.lpr) {
    case 2: SMX_P2T(2); break;
    case 4: SMX_P2T(4); break;
    case 8: SMX_P2T(8); break;
    case 16: SMX_P2T(16); break;
    default: return hipErrorInvalidValue;
    }
#undef SMX_P2T
    return hipGetLastError();
}

hipError_t launch_pass2_tiles(const PassCfg &cfg, const TileView &T, int vk, const float *c, float *x, ColStep cs,
                              const SliceState *st_in, SliceState *st_out, int B, const double *part1, int nparts1,
                              Hist h, hipStream_t s)
{
    if (cfg.grid < 1 || cfg.grid > kMaxPassGrid || nparts1 < 1 || nparts1 > kMaxPassGrid) return hipErrorInvalidValue;
    if (B < 1 || T.ntiles < 1 || T.max_rows < 0 || !tiles_fit(T.max_rows, B)) return hipErrorInvalidValue;
    const bool v8 = cfg.vec == 8;
    if (B > 1) {
        if (vk == VK_F32) return v8 ? pass2_tiles_b<F32U16Tag, 8>(cfg, T, c, x, cs, st_in, st_out, B, part1, nparts1, h, s)
                                    : pass2_tiles_b<F32U16Tag, 4>(cfg, T, c, x, cs, st_in, st_out, B, part1, nparts1, h, s);
        if (vk == VK_BF16P) return v8 ? pass2_tiles_b<Bf16PTag, 8>(cfg, T, c, x, cs, st_in, st_out, B, part1, nparts1, h, s)
                                      : pass2_tiles_b<Bf16PTag, 4>(cfg, T, c, x, cs, st_in, st_out, B, part1, nparts1, h, s);
        if (vk == VK_F16P) return v8 ? pass2_tiles_b<F16PTag, 8>(cfg, T, c, x, cs, st_in, st_out, B, part1, nparts1, h, s)
                                     : pass2_tiles_b<F16PTag, 4>(cfg, T, c, x, cs, st_in, st_out, B, part1, nparts1, h, s);
        return hipErrorInvalidValue;
    }
    if (vk == VK_F32) return v8 ? pass2_tiles<F32U16Tag, 8>(cfg, T, c, x, cs, st_in, st_out, part1, nparts1, h, s)
                                : pass2_tiles<F32U16Tag, 4>(cfg, T, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    if (vk == VK_BF16P) return v8 ? pass2_tiles<Bf16PTag, 8>(cfg, T, c, x, cs, st_in, st_out, part1, nparts1, h, s)
                                  : pass2_tiles<Bf16PTag, 4>(cfg, T, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    if (vk == VK_F16P) return v8 ? pass2_tiles<F16PTag, 8>(cfg, T, c, x, cs, st_in, st_out, part1, nparts1, h, s)
                                 : pass2_tiles<F16PTag, 4>(cfg, T, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    return hipErrorInvalidValue;
}

hipError_t launch_pass2(const PassCfg &cfg, const SpView &At, const RowBlocks &RB, int vk, const float *c, float *x,
                        ColStep cs, const SliceState *st_in, SliceState *st_out, int B, const double *part1,
                        int nparts1, Hist h, hipStream_t s)
{
    if (cfg.grid < 1 || cfg.grid > kMaxPassGrid || nparts1 < 1 || nparts1 > kMaxPassGrid) return hipErrorInvalidValue;
    if (cfg.mode == 3) {
        if (B != 1 || cfg.xlds < 1 || cfg.xlds > kLdsPassFloats) return hipErrorInvalidValue;
        return pass2_lds_kind(cfg, vk, At, c, x, cs, st_in, st_out, part1, nparts1, h, 0, s);
    }
    if (B > 1) {
        if (vk == VK_F32U16) return hipErrorInvalidValue;
        if (vk == VK_F32) return pass2_mm_b<float, 4>(cfg, At, c, x, cs, st_in, st_out, B, part1, nparts1, h, s);
        if (vk == VK_BF16) return pass2_mm_b<Bf16Tag, 8>(cfg, At, c, x, cs, st_in, st_out, B, part1, nparts1, h, s);
        if (vk == VK_BF16P) return pass2_mm_b<Bf16PTag, 4>(cfg, At, c, x, cs, st_in, st_out, B, part1, nparts1, h, s);
        if (vk == VK_F16P) return pass2_mm_b<F16PTag, 4>(cfg, At, c, x, cs, st_in, st_out, B, part1, nparts1, h, s);
        return pass2_mm_b<F16Tag, 8>(cfg, At, c, x, cs, st_in, st_out, B, part1, nparts1, h, s);
    }
    if (cfg.mode == 1) {
        if (vk == VK_F32U16) return pass2_stream<F32U16Tag, 4>(cfg, At, RB, c, x, cs, st_in, st_out, part1, nparts1, h, s);
        if (vk == VK_F32) return pass2_stream<float, 4>(cfg, At, RB, c, x, cs, st_in, st_out, part1, nparts1, h, s);
        if (vk == VK_BF16) return pass2_stream<Bf16Tag, 8>(cfg, At, RB, c, x, cs, st_in, st_out, part1, nparts1, h, s);
        if (vk == VK_BF16P) return pass2_stream<Bf16PTag, 4>(cfg, At, RB, c, x, cs, st_in, st_out, part1, nparts1, h, s);
        if (vk == VK_F16P) return pass2_stream<F16PTag, 4>(cfg, At, RB, c, x, cs, st_in, st_out, part1, nparts1, h, s);
        return pass2_stream<F16Tag, 8>(cfg, At, RB, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    }
    if (vk == VK_BF16P) {
        if (cfg.vec == 8) return pass2_vec<Bf16PTag, 8>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, s);
        return pass2_vec<Bf16PTag, 4>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    }
    if (vk == VK_F16P) {
        if (cfg.vec == 8) return pass2_vec<F16PTag, 8>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, s);
        return pass2_vec<F16PTag, 4>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    }
    if (vk == VK_F32U16) {
        if (cfg.vec == 8) return pass2_vec<F32U16Tag, 8>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, s);
        return pass2_vec<F32U16Tag, 4>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    }
    if (vk == VK_F32) {
        if (cfg.vec == 8) return pass2_vec<float, 8>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, s);
        return pass2_vec<float, 4>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    }
    if (vk == VK_BF16) {
        if (cfg.vec == 8) return pass2_vec<Bf16Tag, 8>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, s);
        return pass2_vec<Bf16Tag, 4>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    }
    if (cfg.vec == 8) return pass2_vec<F16Tag, 8>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, s);
    return pass2_vec<F16Tag, 4>(cfg, At, c, x, cs, st_in, st_out, part1, nparts1, h, s);
}

// Row epilogue of the fused passes with z in LDS (one slice): the row's
// c_i (its step weight times the distance to its band) and its proximity
// term added to pacc; a dose-volume row only stores its value r for the
// ranking and adds nothing here (k_scatter_rows adds its c_i a_i once the
// ranking has set its band).
__device__ inline double fused_epilogue(const RowW &w, long long row, double r, float lo, float up, float d, float sw,
                                        double &pacc)
{
    if (w.dose && row >= w.dose_lo && row < w.dose_hi) {
        w.dose[row - w.dose_lo] = r;
        return 0.0;
    }
    const double t = fmin(fmax(r, (double)lo), (double)up) - r;
    pacc += (double)d * t * t;
    return (double)sw * t;
}

// Fused pass with the gathered vector in LDS.  The plain fused pass gathers
// z_j through the vector memory path once per stored entry, about one
// address per CU per clock, which bounds it on long operators.  Here each
// workgroup (one per CU, 1024 threads) first copies all of z into LDS, beside
// a float32 copy of y (2 x 4n bytes, n up to about 20k), and runs the rows as
// the LDS-staged pass 1 does (LPR lanes per row, four loads of VEC entries in
// flight per lane, rows strided over the grid), gathering from LDS; a row
// outside its band then reads its entries again (from the cache) and adds
// c_i a_i into y with LDS atomics, each group of a wave starting at another
// chunk so that neighbouring rows, which list the same columns in the same
// order, touch different words at once.  y leaves as one float32 partial
// vector per workgroup; k_fused_apply adds them in float64.
template <int LPR, int VEC, typename VT>
__global__ __launch_bounds__(kFusedBlock) void k_fused_zl(SpView A, int n, const float *__restrict__ x,
                                                          const float *__restrict__ lower,
                                                          const float *__restrict__ upper, RowW w,
                                                          const SliceState *__restrict__ st,
                                                          double *__restrict__ partials, float *__restrict__ ypart,
                                                          LinPhase L)
{
    extern __shared__ __align__(16) unsigned char fused_lds[];
    float *zl = reinterpret_cast<float *>(fused_lds);
    float *y = zl + ((n + 3) & ~3);
    __shared__ double lds[kFusedBlock / 64];
    __shared__ double tot[kTrialChunk];
    __shared__ SliceState sS;
    constexpr int RPB = kFusedBlock / LPR;
    constexpr int STEP = LPR * VEC;
    const int lane = threadIdx.x & (LPR - 1);
    const int grp = threadIdx.x / LPR;
    const bool step = L.c && linear_phase<kFusedBlock>(sS, st, L.pp, L.part, 0, L.nparts, tot, L.st_out);
    const bool live = (L.c ? sS.live : st[0].live) != 0;
    for (int j = threadIdx.x; j < n; j += kFusedBlock) y[j] = 0.f;
    double pacc[1] = {0.0};
    if (live) {
        if (step) stage_linear_point<kFusedBlock>(reinterpret_cast<float4 *>(zl), x, L.c, n, sS.s_acc, 1.0 / sS.gn);
        else stage_vector<kFusedBlock>(reinterpret_cast<float4 *>(zl), x, n);
        __syncthreads();
        const long long stride = (long long)gridDim.x * RPB;
        long long row = (long long)blockIdx.x * RPB + grp;
        int beg = 0, end = 0;
        if (row < A.rows) {
            beg = A.ptr[row];
            end = A.ptr[row + 1];
        }
        for (; row < A.rows; row += stride) {
            int nbeg = 0, nend = 0; // the next row's offsets, in flight meanwhile
            if (row + stride < A.rows) {
                nbeg = A.ptr[row + stride];
                nend = A.ptr[row + stride + 1];
            }
            const float lo = lower[row], up = upper[row], d = w.D[row], sw = w.S[row]; // read by every lane
            const double r =
                group_sum<LPR>(row_dot_split<LPR, VEC, VT>(A, beg, end, lane, x, zl, n)) * (double)A.vscale_inv;
            double ct = 0.0;
            if (lane == 0) ct = fused_epilogue(w, row, r, lo, up, d, sw, pacc[0]);
            ct = __shfl(ct, 0, LPR);
            if (ct != 0.0 && end > beg)
                scatter_row<LPR, VEC, VT, float>(A, beg, end, lane, grp, ct * (double)A.vscale_inv, y);
            beg = nbeg;
            end = nend;
        }
    }
    block_sum<1, kFusedBlock>(pacc, lds); // its barriers also order the LDS adds before the copy-out
    if (!live) return;
    if (threadIdx.x == 0) partials[blockIdx.x] = pacc[0];
    float *out = ypart + (long long)blockIdx.x * n;
    for (int j = threadIdx.x; j < n; j += kFusedBlock) out[j] = y[j];
}

// k_fused_zl with each row's first CAP chunks (CAP * LPR * VEC entries) held
// in registers between the dot product and the scatter, so a row outside its
// band adds c_i a_i without reading its entries again: on an operator whose
// rows re-read from the cache outgrow L2, part of those re-reads come from
// HBM.  Within a group, lane l holds the chunk slots of lane (l + group) mod
// LPR (fetch_entries), so neighbouring rows, which list the same columns in
// the same order, hit different LDS addresses in one atomic instruction.
// Entries past CAP chunks are read again as in k_fused_zl.
template <int LPR, int VEC, int CAP, typename VT>
__global__ __launch_bounds__(kFusedBlock) void k_fused_zlr(SpView A, int n, const float *__restrict__ x,
                                                           const float *__restrict__ lower,
                                                           const float *__restrict__ upper, RowW w,
                                                           const SliceState *__restrict__ st,
                                                           double *__restrict__ partials, float *__restrict__ ypart,
                                                           LinPhase L)
{
    extern __shared__ __align__(16) unsigned char fused_lds[];
    float *zl = reinterpret_cast<float *>(fused_lds);
    float *y = zl + ((n + 3) & ~3);
    __shared__ double lds[kFusedBlock / 64];
    __shared__ double tot[kTrialChunk];
    __shared__ SliceState sS;
    constexpr int RPB = kFusedBlock / LPR;
    constexpr int STEP = LPR * VEC;
    const int lane = threadIdx.x & (LPR - 1);
    const int grp = threadIdx.x / LPR;
    const int slot = (lane + grp) & (LPR - 1);
    const bool step = L.c && linear_phase<kFusedBlock>(sS, st, L.pp, L.part, 0, L.nparts, tot, L.st_out);
    const bool live = (L.c ? sS.live : st[0].live) != 0;
    for (int j = threadIdx.x; j < n; j += kFusedBlock) y[j] = 0.f;
    double pacc[1] = {0.0};
    if (live) {
        if (step) stage_linear_point<kFusedBlock>(reinterpret_cast<float4 *>(zl), x, L.c, n, sS.s_acc, 1.0 / sS.gn);
        else stage_vector<kFusedBlock>(reinterpret_cast<float4 *>(zl), x, n);
        __syncthreads();
        const long long stride = (long long)gridDim.x * RPB;
        long long row = (long long)blockIdx.x * RPB + grp;
        int beg = 0, end = 0;
        if (row < A.rows) {
            beg = A.ptr[row];
            end = A.ptr[row + 1];
        }
        for (; row < A.rows; row += stride) {
            // the row's entries, the next row's offsets (in flight while this row
            // is reduced and scattered, so its entries are requested at once) and
            // the epilogue operands: all requested before any of them is used
            EntryRaw<VT, VEC> raw[CAP];
#pragma unroll
            for (int q = 0; q < CAP; ++q) {
                raw[q].zero();
                const int p = beg + (q * LPR + slot) * VEC;
                if (p < end) raw[q].load(A, p);
            }
            int nbeg = 0, nend = 0;
            if (row + stride < A.rows) {
                nbeg = A.ptr[row + stride];
                nend = A.ptr[row + stride + 1];
            }
            const float lo = lower[row], up = upper[row], d = w.D[row], sw = w.S[row]; // read by every lane
            RowRegs<VEC, CAP> R;
#pragma unroll
            for (int q = 0; q < CAP; ++q) raw[q].decode(R.v[q], R.c[q]);
            double acc[2] = {0.0, 0.0};
#pragma unroll
            for (int q = 0; q < CAP; ++q)
#pragma unroll
                for (int e = 0; e < VEC; ++e) // padding slots hold value 0 at column 0
                    acc[q & 1] = fma((double)R.v[q][e], (double)zl[R.c[q][e]], acc[q & 1]);
            const bool tail = end - beg > CAP * STEP;
            if (tail) { // one chunk at a time: the held entries keep most registers
                for (int p = beg + CAP * STEP + lane * VEC; p < end; p += STEP) {
                    float v[VEC];
                    int c[VEC];
                    Entries<VT, VEC>::load(A, p, v, c);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) acc[0] = fma((double)v[e], (double)zl[c[e]], acc[0]);
                }
            }
            const double r = group_sum<LPR>(acc[0] + acc[1]) * (double)A.vscale_inv;
            double ct = 0.0;
            if (lane == 0) ct = fused_epilogue(w, row, r, lo, up, d, sw, pacc[0]);
            ct = __shfl(ct, 0, LPR);
            if (ct != 0.0) {
                const double sc = ct * (double)A.vscale_inv;
#pragma unroll
                for (int q = 0; q < CAP; ++q)
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        if (R.v[q][e] != 0.f) lds_add(&y[R.c[q][e]], sc * (double)R.v[q][e]);
                if (tail) {
                    for (int p = beg + CAP * STEP + lane * VEC; p < end; p += STEP) {
                        float v[VEC];
                        int c[VEC];
                        Entries<VT, VEC>::load(A, p, v, c);
#pragma unroll
                        for (int e = 0; e < VEC; ++e)
                            if (v[e] != 0.f) lds_add(&y[c[e]], sc * (double)v[e]);
                    }
                }
            }
            beg = nbeg;
            end = nend;
        }
    }
    block_sum<1, kFusedBlock>(pacc, lds); // its barriers also order the LDS adds before the copy-out
    if (!live) return;
    if (threadIdx.x == 0) partials[blockIdx.x] = pacc[0];
    float *out = ypart + (long long)blockIdx.x * n;
    for (int j = threadIdx.x; j < n; j += kFusedBlock) out[j] = y[j];
}

// y += sum of c_i a_i over rows [r_lo, r_hi) with c_i already set (the
// dose-volume rows of a problem taking the fused pass, after their ranking):
// one 1024-thread workgroup per CU adds its share of the rows (strided over
// the grid) into an LDS copy of y and leaves it as one float32 partial
// vector, beside the fused pass's own.
template <int LPR, int VEC, typename VT>
__global__ __launch_bounds__(kFusedBlock) void k_scatter_rows(SpView A, int n, long long r_lo, long long r_hi,
                                                              const float *__restrict__ c,
                                                              const SliceState *__restrict__ st,
                                                              float *__restrict__ ypart)
{
    extern __shared__ __align__(16) unsigned char scat_lds[];
    float *y = reinterpret_cast<float *>(scat_lds);
    constexpr int RPB = kFusedBlock / LPR;
    const int lane = threadIdx.x & (LPR - 1);
    const int grp = threadIdx.x / LPR;
    if (st[0].live == 0) return; // the same in every workgroup: the apply reads nothing then
    for (int j = threadIdx.x; j < n; j += kFusedBlock) y[j] = 0.f;
    __syncthreads();
    const long long stride = (long long)gridDim.x * RPB;
    for (long long row = r_lo + (long long)blockIdx.x * RPB + grp; row < r_hi; row += stride) {
        const float ci = c[row];
        const int beg = A.ptr[row], end = A.ptr[row + 1];
        if (ci != 0.f && end > beg)
            scatter_row<LPR, VEC, VT, float>(A, beg, end, lane, grp, (double)ci * (double)A.vscale_inv, y);
    }
    __syncthreads();
    float *out = ypart + (long long)blockIdx.x * n;
    for (int j = threadIdx.x; j < n; j += kFusedBlock) out[j] = y[j];
}

size_t fused_lds_bytes(int64_t n, int acc64) { return size_t(n) * (acc64 ? sizeof(double) : sizeof(float)); }

size_t fused_zl_lds_bytes(int64_t n) { return 2 * size_t((n + 3) & ~int64_t(3)) * sizeof(float); }

int fused_apply_grid(int64_t n) { return (int)grid_for(n, 64, 4096); }

size_t fused_lds_limit()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
    const size_t reserve = 1024; // the fused kernel's own static LDS
    return size_t(v) > reserve ? size_t(v) - reserve : 0;
}

namespace {

struct FusedArgs {
    const SpView *A;
    int64_t n;
    const float *x, *lower, *upper;
    RowW w;
    const SliceState *st;
    double *partials;
    void *ypart;
    LinPhase lp; // lp.c == nullptr: no phase in the pass
};

// prepare != 0: only raise the kernel's dynamic-LDS attribute (done outside
// any stream capture, before the first launch of this shape)
template <int LPR, typename VT, int VEC>
hipError_t fused_zl_go(const FusedCfg &cfg, const FusedArgs &a, int prepare, hipStream_t s)
{
    constexpr int CAP = fused_zl_cap(LPR, VEC);
    if (cfg.cap != 0 && cfg.cap != CAP) return hipErrorInvalidValue;
    auto kern = cfg.cap ? k_fused_zlr<LPR, VEC, CAP, VT> : k_fused_zl<LPR, VEC, VT>;
    const size_t bytes = fused_zl_lds_bytes(a.n);
    if (prepare)
        return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)bytes);
    hipLaunchKernelGGL(kern, dim3(cfg.grid), dim3(kFusedBlock), bytes, s, *a.A, (int)a.n, a.x, a.lower, a.upper, a.w,
                       a.st, a.partials, static_cast<float *>(a.ypart), a.lp);
    return hipGetLastError();
}

template <int LPR, typename VT, int VEC, typename AccT>
hipError_t fused_go(const FusedCfg &cfg, const FusedArgs &a, int prepare, hipStream_t s)
{
    if (cfg.zl) {
        if constexpr (sizeof(AccT) != sizeof(float)) return hipErrorInvalidValue; // float32 partials only
        else return fused_zl_go<LPR, VT, VEC>(cfg, a, prepare, s);
    }
    if (a.lp.c) return hipErrorInvalidValue; // the linear phase rides only on the shapes with z in LDS
    auto kern = k_fused<LPR, VEC, VT, AccT>;
    if (cfg.cap > 0) {
        // register-cached shapes hold CAP*LPR*VEC = 256 entries of a row; with
        // fewer than 16 lanes a row that takes more registers than a lane has
        if constexpr (LPR * VEC >= 64 && LPR >= 16) {
            constexpr int CAP = 256 / (LPR * VEC);
            if (cfg.cap != CAP) return hipErrorInvalidValue;
            kern = k_fused_rc<LPR, VEC, CAP, VT, AccT>;
        } else {
            return hipErrorInvalidValue;
        }
    }
    const size_t bytes = fused_lds_bytes(a.n, sizeof(AccT) == sizeof(double));
    if (prepare)
        return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)bytes);
    hipLaunchKernelGGL(kern, dim3(cfg.grid), dim3(cfg.cap > 0 ? kFusedRcBlock : kFusedBlock), bytes, s, *a.A,
                       (int)a.n, a.x, a.lower, a.upper, a.w, a.st, a.partials, static_cast<AccT *>(a.ypart));
    return hipGetLastError();
}

template <typename VT, int VEC, typename AccT>
hipError_t fused_lpr(const FusedCfg &cfg, const FusedArgs &a, int prepare, hipStream_t s)
{
    switch (cfg.lpr) {
    case 8: return fused_go<8, VT, VEC, AccT>(cfg, a, prepare, s);
    case 16: return fused_go<16, VT, VEC, AccT>(cfg, a, prepare, s);
    case 32: return fused_go<32, VT, VEC, AccT>(cfg, a, prepare, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename VT, int VEC>
hipError_t fused_acc_v(const FusedCfg &cfg, const FusedArgs &a, int prepare, hipStream_t s)
{
    return cfg.acc64 ? fused_lpr<VT, VEC, double>(cfg, a, prepare, s) : fused_lpr<VT, VEC, float>(cfg, a, prepare, s);
}

template <typename VT>
hipError_t fused_acc(const FusedCfg &cfg, const FusedArgs &a, int prepare, hipStream_t s)
{
    if (cfg.vec == 4) return fused_acc_v<VT, 4>(cfg, a, prepare, s);
    if (cfg.vec == 8) return fused_acc_v<VT, 8>(cfg, a, prepare, s);
    return hipErrorInvalidValue;
}

hipError_t fused_dispatch(const FusedCfg &cfg, int vk, const FusedArgs &a, int prepare, hipStream_t s)
{
    if (cfg.grid < 1 || cfg.grid > kMaxPassGrid || a.n < 1 || a.n > (int64_t(1) << 30)) return hipErrorInvalidValue;
    switch (vk) {
    case VK_F32: return fused_acc<float>(cfg, a, prepare, s);
    case VK_BF16: return fused_acc<Bf16Tag>(cfg, a, prepare, s);
    case VK_F16: return fused_acc<F16Tag>(cfg, a, prepare, s);
    case VK_BF16P: return fused_acc<Bf16PTag>(cfg, a, prepare, s);
    case VK_F16P: return fused_acc<F16PTag>(cfg, a, prepare, s);
    case VK_F32U16: return fused_acc<F32U16Tag>(cfg, a, prepare, s);
    default: return hipErrorInvalidValue;
    }
}

} // namespace

hipError_t prepare_fused(const FusedCfg &cfg, int vk, int64_t n)
{
    SpView none{};
    FusedArgs a{&none, n, nullptr, nullptr, nullptr, RowW{nullptr, nullptr, 0}, nullptr, nullptr, nullptr, LinPhase{}};
    return fused_dispatch(cfg, vk, a, 1, nullptr);
}

hipError_t launch_fused(const FusedCfg &cfg, const SpView &A, int vk, int64_t n, const float *x, const float *lower,
                        const float *upper, RowW w, const SliceState *st, double *partials, void *ypart,
                        hipStream_t s, const LinPhase *lp)
{
    if (w.qform) return hipErrorInvalidValue; // the fused pass makes c, never the quadratic form
    if (lp && (!lp->c || !lp->part || !lp->st_out || lp->pp.obj != OBJ_LINEAR || lp->pp.B != 1 || lp->pp.n != n ||
               lp->nparts < 1 || lp->nparts > 65535 || lp->pp.max_trials < 1 || lp->pp.max_trials > 1024 || !cfg.zl))
        return hipErrorInvalidValue;
    FusedArgs a{&A, n, x, lower, upper, w, st, partials, ypart, lp ? *lp : LinPhase{}};
    return fused_dispatch(cfg, vk, a, 0, s);
}

hipError_t launch_fused_apply(const FusedCfg &cfg, int64_t n, const void *ypart, int nvec, float *x, ColStep cs,
                              const SliceState *st_in, SliceState *st_out, const double *part1, Hist h,
                              hipStream_t s, const float *lin_c, double *lin_part, int lin_z)
{
    if (cfg.grid < 1 || cfg.grid > kMaxPassGrid || n < 1 || nvec < cfg.grid || nvec > 2 * cfg.grid ||
        (cfg.acc64 && nvec != cfg.grid) || (lin_part && (!lin_c || cs.defer)) || (lin_z && (!lin_c || cs.defer)))
        return hipErrorInvalidValue;
    const unsigned grid = (unsigned)fused_apply_grid(n);
    if (cfg.acc64)
        hipLaunchKernelGGL(k_fused_apply<double>, dim3(grid), dim3(kApplyBlock), 0, s, static_cast<const double *>(ypart),
                           nvec, (int)n, x, cs, st_in, st_out, part1, cfg.grid, h, lin_c, lin_part, lin_z);
    else
        hipLaunchKernelGGL(k_fused_apply<float>, dim3(grid), dim3(kApplyBlock), 0, s, static_cast<const float *>(ypart),
                           nvec, (int)n, x, cs, st_in, st_out, part1, cfg.grid, h, lin_c, lin_part, lin_z);
    return hipGetLastError();
}

hipError_t launch_lin_partials(const float *x, const float *c, int64_t n, double *part, hipStream_t s)
{
    if (n < 1 || !x || !c || !part) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_lin_partials, dim3((unsigned)fused_apply_grid(n)), dim3(kApplyBlock), 0, s, x, c, (int)n,
                       part);
    return hipGetLastError();
}

namespace {
template <typename VT>
hipError_t scatter_rows_go(int prepare, const SpView &A, int64_t n, long long r_lo, long long r_hi, const float *c,
                           const SliceState *st, float *ypart, int grid, hipStream_t s)
{
    auto kern = k_scatter_rows<8, 4, VT>;
    const size_t bytes = sizeof(float) * size_t(n);
    if (prepare)
        return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)bytes);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kFusedBlock), bytes, s, A, (int)n, r_lo, r_hi, c, st, ypart);
    return hipGetLastError();
}

hipError_t scatter_rows_dispatch(int prepare, const SpView &A, int vk, int64_t n, long long r_lo, long long r_hi,
                                 const float *c, const SliceState *st, float *ypart, int grid, hipStream_t s)
{
    if (n < 1 || (!prepare && (grid < 1 || grid > kMaxPassGrid || r_lo < 0 || r_hi > A.rows || r_lo > r_hi)))
        return hipErrorInvalidValue;
    switch (vk) {
    case VK_F32: return scatter_rows_go<float>(prepare, A, n, r_lo, r_hi, c, st, ypart, grid, s);
    case VK_BF16: return scatter_rows_go<Bf16Tag>(prepare, A, n, r_lo, r_hi, c, st, ypart, grid, s);
    case VK_F16: return scatter_rows_go<F16Tag>(prepare, A, n, r_lo, r_hi, c, st, ypart, grid, s);
    case VK_BF16P: return scatter_rows_go<Bf16PTag>(prepare, A, n, r_lo, r_hi, c, st, ypart, grid, s);
    case VK_F16P: return scatter_rows_go<F16PTag>(prepare, A, n, r_lo, r_hi, c, st, ypart, grid, s);
    case VK_F32U16: return scatter_rows_go<F32U16Tag>(prepare, A, n, r_lo, r_hi, c, st, ypart, grid, s);
    default: return hipErrorInvalidValue;
    }
}
} // namespace

hipError_t prepare_scatter_rows(int vk, int64_t n)
{
    SpView none{};
    return scatter_rows_dispatch(1, none, vk, n, 0, 0, nullptr, nullptr, nullptr, 0, nullptr);
}

hipError_t launch_scatter_rows(const SpView &A, int vk, int64_t n, long long r_lo, long long r_hi, const float *c,
                               const SliceState *st, float *ypart, int grid, hipStream_t s)
{
    return scatter_rows_dispatch(0, A, vk, n, r_lo, r_hi, c, st, ypart, grid, s);
}

hipError_t launch_step_apply(int64_t n, int B, const double *y, float *x, const float *lo, const float *hi,
                             float lambda, int emr, const double *part1, int nparts1, const double *party, int npartsy,
                             const double *partq, int npartsq, const SliceState *st_in, SliceState *st_out, Hist h,
                             hipStream_t s)
{
    if (n < 1 || B < 1 || B > 32 || nparts1 < 1 || npartsy < 1 || (emr && npartsq < 1)) return hipErrorInvalidValue;
    const unsigned grid = grid_for(n * B, kBlock, 2048);
    hipLaunchKernelGGL(k_step_apply, dim3(grid), dim3(kBlock), 0, s, (int)n, B, y, x, lo, hi, lambda, emr, part1,
                       nparts1, party, npartsy, partq, npartsq, st_in, st_out, h);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dose-volume constraints (Section 2.3.3): sets in the output space of the
// split problem (eq. Split).  A constraint owns the rows of one structure;
// "at most k of them above d" (k = floor(V N)) or "at least k at or above d"
// (k = ceil(V N)).  Its nearest point keeps (MAX) or raises to d (MIN) the k
// highest values and lowers the other values above d to d (MAX) or keeps them
// (MIN); as bands, the k highest rows get (-inf, inf) / [d, inf) and the
// others (-inf, d] / (-inf, inf).  Rows rank by the float32-rounded value,
// equal values by row.  Pass 1 stores the rows' values; a radix select over
// 64-bit keys (value bits, then the complement of the row's position) finds
// the k-th highest key; the band kernel then forms c_i and the proximity
// terms, and a one-workgroup kernel per slice adds their sum to pass 1's
// partial 0.  Histogram counts are integers, so their atomic sums are exact.
// ---------------------------------------------------------------------------

__device__ inline int dvc_group(const DvcTable &T, int blk)
{
    int g = 0;
    while (g + 1 < T.n && blk >= T.blk_begin[g + 1]) ++g;
    return g;
}

__device__ inline int dvc_shift(int round) { return round < kDvcRounds - 1 ? 53 - 11 * round : 0; }
__device__ inline int dvc_bits(int round) { return round < kDvcRounds - 1 ? 11 : 9; }

// Order-preserving key of a value rounded to float32 (higher value, higher
// key; -0 counts as +0) with the row's position i in its block.
__device__ inline unsigned long long dvc_key(double r, long long i)
{
    float f = (float)r;
    if (f == 0.0f) f = 0.0f;
    const unsigned u = __float_as_uint(f);
    const unsigned o = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ((unsigned long long)o << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)i);
}

__device__ inline bool dvc_slice_runs(const SliceState *st, int s, int query) { return query || st[s].live != 0; }

// One histogram round: the digit of every candidate key of each constraint
// (round 0: every row, whose key it also stores; later rounds: the keys that
// share the digits fixed so far) into hist[(g * B + s) * kDvcBins + digit].
__global__ __launch_bounds__(kBlock) void k_dvc_hist(DvcTable T, int round, const double *__restrict__ dose,
                                                     unsigned long long *__restrict__ key, unsigned *__restrict__ hist,
                                                     const DvcSel *__restrict__ sel,
                                                     const SliceState *__restrict__ st, int B, int query)
{
    __shared__ unsigned h[kDvcBins];
    const int s = blockIdx.y;
    if (!dvc_slice_runs(st, s, query)) return;
    const int g = dvc_group(T, blockIdx.x);
    const DvcSel S = sel[g * B + s];
    if (round > 0 && S.mode != 0) return;
    for (int b = threadIdx.x; b < kDvcBins; b += kBlock) h[b] = 0u;
    __syncthreads();
    const long long N = T.end[g] - T.begin[g];
    const long long i0 = (long long)(blockIdx.x - T.blk_begin[g]) * kDvcChunk;
    const long long i1 = i0 + kDvcChunk < N ? i0 + kDvcChunk : N;
    const int shift = dvc_shift(round);
    const unsigned mask = (1u << dvc_bits(round)) - 1u;
    const int pshift = shift + dvc_bits(round); // the digits above this round's
    for (long long i = i0 + threadIdx.x; i < i1; i += kBlock) {
        const long long at = (T.begin[g] + i - T.lo) * B + s;
        unsigned long long kk;
        if (round == 0) {
            kk = dvc_key(dose[at], i);
            key[at] = kk;
        } else {
            kk = key[at];
            if ((kk >> pshift) != S.prefix) continue;
        }
        atomicAdd(&h[(unsigned)(kk >> shift) & mask], 1u);
    }
    __syncthreads();
    unsigned *H = hist + (size_t)(g * B + s) * kDvcBins;
    for (int b = threadIdx.x; b < kDvcBins; b += kBlock)
        if (h[b]) atomicAdd(&H[b], h[b]);
}

// One workgroup per constraint and slice: the digit that holds the k-th
// highest key among the candidates, from the highest digit down; then the
// histogram is cleared for the next round.  The selection ends once every
// candidate of that digit ranks high (or after the last round, where a digit
// holds one key).
__global__ __launch_bounds__(kBlock) void k_dvc_pick(DvcTable T, int round, unsigned *__restrict__ hist,
                                                     DvcSel *__restrict__ sel, const SliceState *__restrict__ st,
                                                     int B, int query)
{
    __shared__ unsigned long long suf[kBlock];
    const int g = blockIdx.x, s = blockIdx.y;
    if (!dvc_slice_runs(st, s, query)) return;
    DvcSel *S = sel + (g * B + s);
    if (round > 0 && S->mode != 0) return;
    unsigned *H = hist + (size_t)(g * B + s) * kDvcBins;
    constexpr int PER = kDvcBins / kBlock;
    const long long N = T.end[g] - T.begin[g], k = T.k[g];
    unsigned cnt[PER];
    unsigned long long tsum = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        cnt[j] = H[threadIdx.x * PER + j];
        tsum += cnt[j];
    }
    if (round == 0 && (k <= 0 || k >= N)) {
        if (threadIdx.x == 0) {
            S->mode = k <= 0 ? 1 : 3;
            S->prefix = 0;
            S->thr = 0;
            S->krem = 0;
        }
    } else {
        const long long krem = round == 0 ? k : S->krem;
        const unsigned long long prefix = round == 0 ? 0ull : S->prefix;
        // suffix sums over threads: suf[t] = counts of bins >= t * PER
        suf[threadIdx.x] = tsum;
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {
            const unsigned long long v = suf[threadIdx.x] + (threadIdx.x + off < kBlock ? suf[threadIdx.x + off] : 0ull);
            __syncthreads();
            suf[threadIdx.x] = v;
            __syncthreads();
        }
        const long long incl = (long long)suf[threadIdx.x], excl = incl - (long long)tsum;
        if (excl < krem && krem <= incl) {
            long long above = excl;
            int dig = threadIdx.x * PER;
            long long kr = 0;
            unsigned c_dig = 0;
            for (int j = PER - 1; j >= 0; --j) {
                if (above + (long long)cnt[j] >= krem) {
                    dig = threadIdx.x * PER + j;
                    kr = krem - above;
                    c_dig = cnt[j];
                    break;
                }
                above += cnt[j];
            }
            const unsigned long long np = (prefix << dvc_bits(round)) | (unsigned long long)dig;
            if ((long long)c_dig == kr || round == kDvcRounds - 1) {
                S->mode = 2;
                S->thr = np << dvc_shift(round);
            } else {
                S->mode = 0;
                S->prefix = np;
                S->krem = kr;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) H[threadIdx.x * PER + j] = 0u;
}

// The bands the selection gives, c_i = S_i t_i and per-workgroup partials of
// the proximity terms D_i t_i^2 in epart[s * nblk + workgroup].
__global__ __launch_bounds__(kBlock) void k_dvc_bands(DvcTable T, const double *__restrict__ dose,
                                                      const unsigned long long *__restrict__ key,
                                                      const DvcSel *__restrict__ sel, const float *__restrict__ D,
                                                      const float *__restrict__ Sw, float *__restrict__ c,
                                                      double *__restrict__ epart, const SliceState *__restrict__ st,
                                                      int B, int query)
{
    __shared__ double lds[4];
    const int s = blockIdx.y;
    if (!dvc_slice_runs(st, s, query)) return;
    const int g = dvc_group(T, blockIdx.x);
    const DvcSel S = sel[g * B + s];
    const long long N = T.end[g] - T.begin[g];
    const long long i0 = (long long)(blockIdx.x - T.blk_begin[g]) * kDvcChunk;
    const long long i1 = i0 + kDvcChunk < N ? i0 + kDvcChunk : N;
    const double dref = T.dose[g];
    const bool upper_kind = T.sense[g] == 0;
    double pacc[1] = {0.0};
    for (long long i = i0 + threadIdx.x; i < i1; i += kBlock) {
        const long long row = T.begin[g] + i;
        const long long at = (row - T.lo) * B + s;
        const double r = dose[at];
        const bool high = S.mode == 3 || (S.mode == 2 && key[at] >= S.thr);
        double lo = -INFINITY, up = INFINITY;
        if (upper_kind) {
            if (!high) up = dref;
        } else if (high) {
            lo = dref;
        }
        const double t = fmin(fmax(r, lo), up) - r;
        c[row * B + s] = (float)((double)Sw[row] * t);
        pacc[0] += (double)D[row] * t * t;
    }
    block_sum<1>(pacc, lds);
    if (threadIdx.x == 0) epart[(long long)s * T.nblk + blockIdx.x] = pacc[0];
}

// Adds the band kernel's partials of slice s (summed in workgroup order) to
// pass 1's partial 0 of that slice.
__global__ __launch_bounds__(kBlock) void k_dvc_fold(const double *__restrict__ epart, int nblk,
                                                     double *__restrict__ part1, int nparts1,
                                                     const SliceState *__restrict__ st, int query)
{
    __shared__ double lds[4];
    const int s = blockIdx.x;
    if (!dvc_slice_runs(st, s, query)) return;
    double tot[1];
    sum_slots<1>(epart, (long long)s * nblk, nblk, tot, lds);
    if (threadIdx.x == 0) part1[(long long)s * nparts1] += tot[0];
}

hipError_t launch_dvc(const DvcTable &T, const double *dose, unsigned long long *key, unsigned *hist, DvcSel *sel,
                      const float *D, const float *S, float *c, double *epart, double *part1, int nparts1,
                      const SliceState *st, int B, int query, hipStream_t s)
{
    if (T.n < 1 || T.n > kMaxDvc || T.nblk < 1 || B < 1 || B > 32) return hipErrorInvalidValue;
    const dim3 blk(kBlock), gall(T.nblk, B), gsel(T.n, B);
    for (int r = 0; r < kDvcRounds; ++r) {
        hipLaunchKernelGGL(k_dvc_hist, gall, blk, 0, s, T, r, dose, key, hist, sel, st, B, query);
        hipLaunchKernelGGL(k_dvc_pick, gsel, blk, 0, s, T, r, hist, sel, st, B, query);
    }
    hipLaunchKernelGGL(k_dvc_bands, gall, blk, 0, s, T, dose, key, sel, D, S, c, epart, st, B, query);
    hipLaunchKernelGGL(k_dvc_fold, dim3(B), blk, 0, s, epart, T.nblk, part1, nparts1, st, query);
    return hipGetLastError();
}


hipError_t launch_query_prox(SliceState *st, int B, const double *partials, int nparts, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_query_prox, dim3(1), dim3(kBlock), 0, s, st, B, partials, nparts, out);
    return hipGetLastError();
}

hipError_t launch_phase(const PertParams &pp, const float *x, float *g, const float *lin_c, const SliceState *st,
                        int eval_only, double *partials, hipStream_t s)
{
    const dim3 grid(phase_grid(pp), pp.B), block(kBlock);
    if (pp.obj == OBJ_TV2D)
        hipLaunchKernelGGL(k_phase_tv, grid, block, 0, s, x, g, st, pp, eval_only, partials);
    else
        hipLaunchKernelGGL(k_phase_flat, grid, block, 0, s, x, g, lin_c, st, pp, eval_only, partials);
    return hipGetLastError();
}

hipError_t launch_eval_objective(SliceState *st, const PertParams &pp, const double *partials, double *out,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(k_eval_objective, dim3(1), dim3(kBlock), 0, s, st, pp, partials, phase_grid(pp), out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Variance stopping rule (Section 2.3.2): omega_k = ||x^k - x^{k-1}|| / ||x^k||
// (0 when x^k = 0); the run stops once the sample variance of omega_1 ..
// omega_k (k >= 2) is below the threshold.  Running mean and sum of squared
// deviations (Welford), in float64, per slice.
// ---------------------------------------------------------------------------

__global__ void k_copy(float *__restrict__ dst, const float *__restrict__ src, long long count)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Per-workgroup partials of ||x - xprev||^2 and ||x||^2 for every slice:
// partials[(s * grid + block) * 2 + {0, 1}].
__global__ __launch_bounds__(kBlock) void k_iter_norms(const float *__restrict__ x, const float *__restrict__ xprev,
                                                       long long n, int B, double *__restrict__ partials)
{
    __shared__ double lds[4 * 2];
    for (int s = 0; s < B; ++s) {
        double v[2] = {0.0, 0.0};
        for (long long j = (long long)blockIdx.x * kBlock + threadIdx.x; j < n; j += (long long)gridDim.x * kBlock) {
            const double a = (double)x[j * B + s], b = (double)xprev[j * B + s];
            v[0] += (a - b) * (a - b);
            v[1] += a * a;
        }
        block_sum<2>(v, lds);
        if (threadIdx.x == 0) {
            partials[((long long)s * gridDim.x + blockIdx.x) * 2 + 0] = v[0];
            partials[((long long)s * gridDim.x + blockIdx.x) * 2 + 1] = v[1];
        }
    }
}

// One workgroup: updates the statistics of the slices that ran the iteration
// just ended and stops those whose variance fell below the threshold (a
// reason already set by the proximity rules takes precedence).  In place on
// the current state buffer (no other workgroup touches it in this launch).
__global__ __launch_bounds__(kBlock) void k_stop_var(SliceState *__restrict__ st, int B,
                                                     const double *__restrict__ partials, int nparts)
{
    __shared__ double lds[4 * 2];
    for (int s = 0; s < B; ++s) {
        double tot[2];
        sum_slots<2>(partials, (long long)s * nparts, nparts, tot, lds);
        if (threadIdx.x == 0) {
            SliceState S = st[s];
            if (S.ran && S.stop_on && S.stop_var > 0.0) {
                const double om = tot[1] > 0.0 ? sqrt(tot[0]) / sqrt(tot[1]) : 0.0;
                S.var_n += 1.0;
                const double delta = om - S.var_mean;
                S.var_mean += delta / S.var_n;
                S.var_m2 += delta * (om - S.var_mean);
                if (S.stop_reason == STOP_NONE && S.var_n >= 2.0 && S.var_m2 / (S.var_n - 1.0) < S.stop_var)
                    S.stop_reason = STOP_VAR;
                S.live = slice_runs(S);
                st[s] = S;
            }
        }
    }
}

hipError_t launch_copy(float *dst, const float *src, int64_t count, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy, dim3(grid_for(count, kBlock, 4096)), dim3(kBlock), 0, s, dst, src, (long long)count);
    return hipGetLastError();
}

hipError_t launch_iter_norms(const float *x, const float *xprev, int64_t n, int B, double *partials, int *nparts,
                             hipStream_t s)
{
    const unsigned grid = grid_for(n, kBlock, 256);
    *nparts = (int)grid;
    hipLaunchKernelGGL(k_iter_norms, dim3(grid), dim3(kBlock), 0, s, x, xprev, (long long)n, B, partials);
    return hipGetLastError();
}

hipError_t launch_stop_var(SliceState *st, int B, const double *partials, int nparts, hipStream_t s)
{
    hipLaunchKernelGGL(k_stop_var, dim3(1), dim3(kBlock), 0, s, st, B, partials, nparts);
    return hipGetLastError();
}

bool phase_in_one_launch(const PertParams &pp)
{
    return (pp.obj == OBJ_SQNORM || pp.obj == OBJ_L1 || pp.obj == OBJ_LINEAR) && pp.n >= 1 &&
           pp.n <= kSmallPhaseMaxN;
}

static size_t phase_small_lds(const PertParams &pp) { return 2 * sizeof(float) * size_t(pp.n); }

hipError_t prepare_phase_small()
{
    // the largest size any problem asks for: the attribute is the kernel's, not a problem's
    const int bytes = (int)(2 * sizeof(float) * kSmallPhaseMaxN);
    for (const void *k : {reinterpret_cast<const void *>(k_phase_small<OBJ_SQNORM>),
                          reinterpret_cast<const void *>(k_phase_small<OBJ_L1>),
                          reinterpret_cast<const void *>(k_phase_small<OBJ_LINEAR>)}) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_phase_small(const PertParams &pp, float *x, const float *lin_c, const SliceState *st_in,
                              SliceState *st_out, hipStream_t s)
{
    if (!phase_in_one_launch(pp) || pp.max_trials < 1 || pp.max_trials > 1024 || pp.B < 1) return hipErrorInvalidValue;
    const dim3 grid(1, pp.B), block(kSmallPhaseBlock);
    const size_t lds = phase_small_lds(pp);
    if (pp.obj == OBJ_SQNORM)
        hipLaunchKernelGGL(k_phase_small<OBJ_SQNORM>, grid, block, lds, s, x, lin_c, st_in, st_out, pp);
    else if (pp.obj == OBJ_L1)
        hipLaunchKernelGGL(k_phase_small<OBJ_L1>, grid, block, lds, s, x, lin_c, st_in, st_out, pp);
    else
        hipLaunchKernelGGL(k_phase_small<OBJ_LINEAR>, grid, block, lds, s, x, lin_c, st_in, st_out, pp);
    return hipGetLastError();
}

hipError_t launch_trial_linear(const PertParams &pp, float *x, const float *c, const SliceState *st_in,
                               SliceState *st_out, const double *part_phase, hipStream_t s, int nt)
{
    if (pp.obj != OBJ_LINEAR || pp.max_trials < 1 || pp.max_trials > 1024) return hipErrorInvalidValue;
    if (nt == 0) nt = phase_grid(pp); // the direction launch's partials
    if (nt < 1 || nt > 65535 || (nt != phase_grid(pp) && pp.B != 1)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_trial_linear, dim3(nt, pp.B), dim3(kBlock), 0, s, x, c, st_in, st_out, pp, part_phase);
    return hipGetLastError();
}

hipError_t launch_trial_close(const PertParams &pp, float *x, const float *g, const SliceState *st_in,
                              SliceState *st_out, const double *part_prev, hipStream_t s)
{
    if (pp.max_trials < 1 || pp.max_trials > 1024) return hipErrorInvalidValue;
    const long long g_need = (pp.n + kTrialBlock - 1) / kTrialBlock; // one unknown a thread, at most 256 workgroups
    const unsigned grid = (unsigned)std::max(1LL, std::min(g_need, 256LL));
    hipLaunchKernelGGL(k_trial_close, dim3(grid, pp.B), dim3(kTrialBlock), 0, s, x, g, st_in, st_out, pp,
                       (int)phase_grid(pp), part_prev);
    return hipGetLastError();
}

hipError_t launch_trial(const PertParams &pp, float *x, const float *g, const SliceState *st_in, SliceState *st_out,
                        int first, int evaluate, const double *part_prev, double *part_out, hipStream_t s)
{
    if (pp.max_trials < 1 || pp.max_trials > 1024) return hipErrorInvalidValue;
    const dim3 grid(phase_grid(pp), pp.B), block(kBlock);
    if (pp.obj == OBJ_TV2D)
        hipLaunchKernelGGL(k_trial_tv, grid, dim3(kTrialBlock), 0, s, x, g, st_in, st_out, pp, first, evaluate,
                           part_prev, part_out);
    else
        hipLaunchKernelGGL(k_trial_flat, grid, block, 0, s, x, g, st_in, st_out, pp, first, evaluate, part_prev,
                           part_out);
    return hipGetLastError();
}

} // namespace smx
