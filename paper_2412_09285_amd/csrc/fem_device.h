// Device helpers shared by the step kernels (fem_kernels.hip, fem_manip.hip):
// bfloat16 conversion, vector loads and stores of the state and the marginal
// copy, the optimiser update, fixed-point column sums, the Max-k-SAT marginal
// encoding, and the team / workgroup reductions.
#pragma once

#include "fem_internal.h"

namespace fem {

// ---------------------------------------------------------------- helpers --
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// round-to-nearest-even float -> bfloat16 (NaN kept quiet)
__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// V consecutive float32 values
template <int V>
__device__ __forceinline__ void ld_f32(const float* __restrict__ p, float (&x)[V])
{
    if constexpr (V == 1) {
        x[0] = p[0];
    } else if constexpr (V == 2) {
        f32x2 t = *reinterpret_cast<const f32x2*>(p);
        x[0] = t.x; x[1] = t.y;
    } else {
#pragma unroll
        for (int k = 0; k < V / 4; ++k) {
            f32x4 t = reinterpret_cast<const f32x4*>(p)[k];
            x[4 * k] = t.x; x[4 * k + 1] = t.y; x[4 * k + 2] = t.z; x[4 * k + 3] = t.w;
        }
    }
}

template <int V>
__device__ __forceinline__ void st_f32(float* __restrict__ p, const float (&x)[V])
{
    if constexpr (V == 1) {
        p[0] = x[0];
    } else if constexpr (V == 2) {
        f32x2 t; t.x = x[0]; t.y = x[1];
        *reinterpret_cast<f32x2*>(p) = t;
    } else {
#pragma unroll
        for (int k = 0; k < V / 4; ++k) {
            f32x4 t; t.x = x[4 * k]; t.y = x[4 * k + 1]; t.z = x[4 * k + 2]; t.w = x[4 * k + 3];
            reinterpret_cast<f32x4*>(p)[k] = t;
        }
    }
}

// V consecutive bfloat16 values, widened
template <int V>
__device__ __forceinline__ void ld_bf16(const uint16_t* __restrict__ p, float (&x)[V])
{
    if constexpr (V == 1) {
        x[0] = bf16_to_f32(p[0]);
    } else if constexpr (V == 2) {
        uint32_t t = *reinterpret_cast<const uint32_t*>(p);
        x[0] = __uint_as_float(t << 16); x[1] = __uint_as_float(t & 0xffff0000u);
    } else if constexpr (V == 4) {
        u32x2 t = *reinterpret_cast<const u32x2*>(p);
        x[0] = __uint_as_float(t.x << 16); x[1] = __uint_as_float(t.x & 0xffff0000u);
        x[2] = __uint_as_float(t.y << 16); x[3] = __uint_as_float(t.y & 0xffff0000u);
    } else {
#pragma unroll
        for (int k = 0; k < V / 8; ++k) {
            u32x4 t = reinterpret_cast<const u32x4*>(p)[k];
            x[8 * k + 0] = __uint_as_float(t.x << 16); x[8 * k + 1] = __uint_as_float(t.x & 0xffff0000u);
            x[8 * k + 2] = __uint_as_float(t.y << 16); x[8 * k + 3] = __uint_as_float(t.y & 0xffff0000u);
            x[8 * k + 4] = __uint_as_float(t.z << 16); x[8 * k + 5] = __uint_as_float(t.z & 0xffff0000u);
            x[8 * k + 6] = __uint_as_float(t.w << 16); x[8 * k + 7] = __uint_as_float(t.w & 0xffff0000u);
        }
    }
}

template <int V>
__device__ __forceinline__ void st_bf16(uint16_t* __restrict__ p, const float (&x)[V])
{
    if constexpr (V == 1) {
        p[0] = f32_to_bf16(x[0]);
    } else if constexpr (V == 2) {
        *reinterpret_cast<uint32_t*>(p) = (uint32_t)f32_to_bf16(x[0]) | ((uint32_t)f32_to_bf16(x[1]) << 16);
    } else if constexpr (V == 4) {
        u32x2 t;
        t.x = (uint32_t)f32_to_bf16(x[0]) | ((uint32_t)f32_to_bf16(x[1]) << 16);
        t.y = (uint32_t)f32_to_bf16(x[2]) | ((uint32_t)f32_to_bf16(x[3]) << 16);
        *reinterpret_cast<u32x2*>(p) = t;
    } else {
#pragma unroll
        for (int k = 0; k < V / 8; ++k) {
            u32x4 t;
            t.x = (uint32_t)f32_to_bf16(x[8 * k + 0]) | ((uint32_t)f32_to_bf16(x[8 * k + 1]) << 16);
            t.y = (uint32_t)f32_to_bf16(x[8 * k + 2]) | ((uint32_t)f32_to_bf16(x[8 * k + 3]) << 16);
            t.z = (uint32_t)f32_to_bf16(x[8 * k + 4]) | ((uint32_t)f32_to_bf16(x[8 * k + 5]) << 16);
            t.w = (uint32_t)f32_to_bf16(x[8 * k + 6]) | ((uint32_t)f32_to_bf16(x[8 * k + 7]) << 16);
            reinterpret_cast<u32x4*>(p)[k] = t;
        }
    }
}

template <typename MT, int V>
__device__ __forceinline__ void ld_marg(const MT* p, float (&x)[V])
{
    if constexpr (sizeof(MT) == 4) ld_f32<V>(reinterpret_cast<const float*>(p), x);
    else ld_bf16<V>(reinterpret_cast<const uint16_t*>(p), x);
}

template <typename MT, int V>
__device__ __forceinline__ void st_marg(MT* p, const float (&x)[V])
{
    if constexpr (sizeof(MT) == 4) st_f32<V>(reinterpret_cast<float*>(p), x);
    else st_bf16<V>(reinterpret_cast<uint16_t*>(p), x);
}

// h, m1, m2 are read once and written once per step: with NT the accesses
// are non-temporal, so they do not evict the gathered marginal copy from L2
// and the Infinity Cache.
template <int V, bool NT>
__device__ __forceinline__ void ld_state(const float* __restrict__ p, float (&x)[V])
{
    if constexpr (!NT || V < 4) {
        if constexpr (NT && V == 1) x[0] = __builtin_nontemporal_load(p);
        else if constexpr (NT && V == 2) {
            f32x2 t = __builtin_nontemporal_load(reinterpret_cast<const f32x2*>(p));
            x[0] = t.x; x[1] = t.y;
        } else ld_f32<V>(p, x);
    } else {
#pragma unroll
        for (int k = 0; k < V / 4; ++k) {
            f32x4 t = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p) + k);
            x[4 * k] = t.x; x[4 * k + 1] = t.y; x[4 * k + 2] = t.z; x[4 * k + 3] = t.w;
        }
    }
}

template <int V, bool NT>
__device__ __forceinline__ void st_state(float* __restrict__ p, const float (&x)[V])
{
    if constexpr (!NT || V < 4) {
        if constexpr (NT && V == 1) __builtin_nontemporal_store(x[0], p);
        else if constexpr (NT && V == 2) {
            f32x2 t; t.x = x[0]; t.y = x[1];
            __builtin_nontemporal_store(t, reinterpret_cast<f32x2*>(p));
        } else st_f32<V>(p, x);
    } else {
#pragma unroll
        for (int k = 0; k < V / 4; ++k) {
            f32x4 t; t.x = x[4 * k]; t.y = x[4 * k + 1]; t.z = x[4 * k + 2]; t.w = x[4 * k + 3];
            __builtin_nontemporal_store(t, reinterpret_cast<f32x4*>(p) + k);
        }
    }
}

// ------------------------------------------------------------- fast math --
// The step kernels are bound by their vector ALU, not by memory, once the
// neighbour gathers hit L2: the general-purpose expf / tanhf / log1pf and
// IEEE divisions cost tens of instructions each.  These forms use the
// hardware base-2 exponential and logarithm, reciprocal and square root
// (about 1 ulp each) with the corrections below, a few ulp in all; the
// gradient's cancellation-prone combination stays in double in the callers.

// exp(-a), a >= 0 (any a): 2^t with t = -a log2(e) rounded, and the rounding
// error of t (exact product error by fma, plus the low part of log2(e))
// applied as the first-order factor 1 + c ln 2
__device__ __forceinline__ float exp_neg(float a)
{
    constexpr float L2E = 1.44269502162933349609375f;      // float(log2 e)
    constexpr float L2E_LO = 1.925963033500011e-08f;       // log2 e - L2E
    constexpr float LN2 = 0.693147180559945309f;
    const float t = -a * L2E;
    const float c = fmaf(-a, L2E_LO, fmaf(-a, L2E, -t));
    const float e0 = __builtin_amdgcn_exp2f(t);
    return fmaf(e0, c * LN2, e0);
}

__device__ __forceinline__ float rcp_f(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt_f(float x) { return __builtin_amdgcn_sqrtf(x); }

// tanh(y / 2): the odd Taylor series of tanh(z), z = |y|/2, up to z^11 where
// |y| < 0.55 (truncation below 1e-9 relative), else (1 - e)/(1 + e) with
// e = exp(-|y|), where 1 - e >= 0.42 keeps its relative precision; the sign
// of y restored
__device__ __forceinline__ float tanh_half(float y)
{
    const float a = fabsf(y);
    const float z = 0.5f * a, z2 = z * z;
    float p = fmaf(z2, 21844.0f / 6081075.0f, -1382.0f / 155925.0f);
    p = fmaf(p, z2, 62.0f / 2835.0f);
    p = fmaf(p, z2, -17.0f / 315.0f);
    p = fmaf(p, z2, 2.0f / 15.0f);
    p = fmaf(p, z2, -1.0f / 3.0f);
    const float small = fmaf(p * z2, z, z);
    const float e = exp_neg(a);
    const float large = (1.0f - e) * rcp_f(1.0f + e);
    return copysignf(a < 0.55f ? small : large, y);
}

// ln(1 + e) for e >= 0: u = 1 + e rounded, then ln(u) e / (u - 1) (the
// quotient cancels the rounding of u); e itself where u rounds to 1
__device__ __forceinline__ float log1p_f(float e)
{
    constexpr float LN2 = 0.693147180559945309f;
    const float u = 1.0f + e;
    const float d = u - 1.0f;
    const float l = __builtin_amdgcn_logf(u) * LN2;
    return d == 0.0f ? e : l * (e * rcp_f(d));
}

// For one logit h with e = exp(-|h|) and r = 1/(1+e): the smaller of P and
// 1 - P is e r, and P(1 - P) = e r^2, both without cancellation.

// The optimiser step, torch.optim semantics (a uniform branch):
//  Adam:    g += wd h; m1 = b1 m1 + (1-b1) g; m2 = b2 m2 + (1-b2) g^2;
//           h -= step_size * m1 / (sqrt(m2)/sqrt(1-b2^n) + eps)
//  RMSprop: g += wd h; m2 = a m2 + (1-a) g^2; d = sqrt(m2) + eps;
//           momentum > 0: m1 = mu m1 + g/d, h -= lr m1;  else h -= lr g/d
//  SGD:     g += wd h; momentum != 0: m1 = g (first step) or mu m1 + (1-damp) g,
//           g = m1;  h -= lr g
// (the divisions by the bias correction and the denominator are taken as
// products with a reciprocal: 1/sqrt(1 - b2^n) comes from the host in double)
__device__ __forceinline__ float adam_update(float x, float g, float& m1, float& m2, const StepScalars& s)
{
    g = fmaf(s.wd, x, g);
    if (s.opt == 0) {
        m1 = fmaf(s.b1, m1, s.one_m_b1 * g);
        m2 = fmaf(s.b2, m2, s.one_m_b2 * (g * g));
        const float denom = fmaf(sqrt_f(m2), s.inv_bc2_sqrt, s.eps);
        return fmaf(-s.step_size, m1 * rcp_f(denom), x);
    }
    if (s.opt == 1) {
        m2 = fmaf(s.rms_alpha, m2, s.one_m_rms * (g * g));
        const float id = rcp_f(sqrt_f(m2) + s.eps);
        if (s.mom > 0.0f) {
            m1 = fmaf(s.mom, m1, g * id);
            return fmaf(-s.lr, m1, x);
        }
        return fmaf(-s.lr, g * id, x);
    }
    if (s.mom != 0.0f) {
        m1 = s.first ? g : fmaf(s.mom, m1, (1.0f - s.damp) * g);
        g = m1;
    }
    return fmaf(-s.lr, g, x);
}

// 2^-40 fixed point of a probability in [0, 1]
__device__ __forceinline__ long long to_fixed(double p) { return (long long)rint(p * 1099511627776.0); }

// rint(x) as an integer for 0 <= x < 2^51: x + 1.5 * 2^52 has a unit ulp, so
// its low mantissa bits hold x rounded to the nearest integer (ties to even)
__device__ __forceinline__ long long rint_small_i64(double x)
{
    return (long long)__double_as_longlong(x + 6755399441055744.0) - 0x4338000000000000LL;
}

// exp(d) in double for d <= 0, to about 1e-13 relative: t = d log2(e) =
// k + f with k = rint(t), and e^(f ln 2), |f ln 2| <= 0.35, by its Taylor
// polynomial to the 12th power (truncation below 1e-15); large |d| underflow
// to 0 through the exponent
__device__ __forceinline__ double exp_dp_neg(double d)
{
    const double t = d * 1.4426950408889634;
    const double k = rint(t);
    const double y = (t - k) * 0.6931471805599453;
    double p = 1.0 / 479001600.0;   // 1/12!
    p = fma(p, y, 1.0 / 39916800.0);
    p = fma(p, y, 1.0 / 3628800.0);
    p = fma(p, y, 1.0 / 362880.0);
    p = fma(p, y, 1.0 / 40320.0);
    p = fma(p, y, 1.0 / 5040.0);
    p = fma(p, y, 1.0 / 720.0);
    p = fma(p, y, 1.0 / 120.0);
    p = fma(p, y, 1.0 / 24.0);
    p = fma(p, y, 1.0 / 6.0);
    p = fma(p, y, 0.5);
    p = fma(p, y, 1.0);
    p = fma(p, y, 1.0);
    return ldexp(p, (int)fmax(k, -2000.0));
}

// The softmax of one replica's q fields in double: the float marginals P
// (rounded from the double values) and their column-sum contributions in
// 2^-40 fixed point, vw P per state (vw the node weight).  Double, because the
// sum over all nodes of float32 marginals would carry their rounding into the
// global balance term.
template <int Q>
__device__ __forceinline__ void softmax_colsum(const float (&h)[Q], long long (&cs)[Q], double vw, float (&P)[Q])
{
    float mx = h[0];
#pragma unroll
    for (int s = 1; s < Q; ++s) mx = fmaxf(mx, h[s]);
    double e[Q], Z = 0.0;
#pragma unroll
    for (int s = 0; s < Q; ++s) {
        e[s] = exp_dp_neg((double)h[s] - (double)mx);
        Z += e[s];
    }
    const double iz = 1.0 / Z;
    const bool unit = vw == 1.0;
#pragma unroll
    for (int s = 0; s < Q; ++s) {
        const double p = e[s] * iz;
        P[s] = (float)p;
        // unit weights: p 2^40 < 2^51, the cheap rounding applies
        cs[s] += unit ? rint_small_i64(p * 1099511627776.0) : to_fixed(vw * p);
    }
}


// Max-k-SAT stored marginal: the smaller of P(x=1) and P(x=0), negative (sign
// bit set) when P(x=1) > 1/2.  Both tails keep full relative precision.
__device__ __forceinline__ float sat_encode(float h)
{
    const float e = exp_neg(fabsf(h));
    const float small = e * rcp_f(1.0f + e);
    return h > 0.0f ? -small : small;
}
// probability that a literal of polarity pos is false, from the stored value
__device__ __forceinline__ float sat_u(float s, bool pos)
{
    bool hi = signbit(s);
    float a = fabsf(s);
    return (pos == hi) ? a : 1.0f - a;
}
// the same with the polarity as a sign-bit mask (SAT_POS or 0): flipping the
// stored sign for a positive literal leaves u = s' where s' >= +0, and
// u = 1 + s' where the sign bit of s' is set
__device__ __forceinline__ float sat_u_bits(float s, uint32_t pos_mask)
{
    const uint32_t b = __float_as_uint(s) ^ pos_mask;
    const float sp = __uint_as_float(b);
    return (b & 0x80000000u) ? 1.0f + sp : sp;
}

// Butterfly over the teams of one wave (lanes that hold the same replicas),
// then a fixed-order sum over the waves of the workgroup.  vals[k] are per-lane
// values, K per lane.  Results land in out[k * L * Vl + lane * Vl + v]-style
// layout chosen by the caller through 'store'.
template <typename T, int K>
__device__ __forceinline__ void team_butterfly(T (&v)[K], int lanes_log2)
{
    for (int off = 1 << lanes_log2; off < 64; off <<= 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += __shfl_xor(v[k], off, 64);
    }
}

// ------------------------------------------------------- geometry helpers --
// Block -> (tile, replica segment).  Tile-major grids are (n_tiles, nseg);
// segment-major grids are (nseg, n_tiles), so that consecutive workgroups,
// which the dispatcher deals round-robin to the eight XCDs, take different
// replica segments of the same rows and each XCD's L2 serves the gathers of
// one segment's columns.
__device__ __forceinline__ int blk_tile(int seg_major) { return seg_major ? blockIdx.y : blockIdx.x; }
__device__ __forceinline__ int blk_seg(int seg_major) { return seg_major ? blockIdx.x : blockIdx.y; }

struct TeamIdx {
    int lane, wave, nwaves, L, tl, team, teams;
};
__device__ __forceinline__ TeamIdx team_idx(int lanes_log2)
{
    TeamIdx t;
    t.lane = threadIdx.x & 63;
    t.wave = threadIdx.x >> 6;
    t.nwaves = blockDim.x >> 6;
    t.L = 1 << lanes_log2;
    t.tl = t.lane & (t.L - 1);
    t.team = t.wave * (64 >> lanes_log2) + (t.lane >> lanes_log2);
    t.teams = t.nwaves * (64 >> lanes_log2);
    return t;
}

// Sum K per-lane values over the workgroup's teams in a fixed order (butterfly
// within the wave, then waves in order) and hand each total to store(k, l, s),
// where l is the lane-in-team index.  lds must hold nwaves * L * K values.
template <typename T, int K, typename Store>
__device__ __forceinline__ void block_reduce_store(T (&v)[K], const TeamIdx& ti, int lanes_log2, T* lds,
                                                   Store store)
{
    team_butterfly<T, K>(v, lanes_log2);
    if (ti.lane < ti.L) {
#pragma unroll
        for (int k = 0; k < K; ++k) lds[(ti.wave * K + k) * ti.L + ti.lane] = v[k];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ti.L * K; t += blockDim.x) {
        const int k = t / ti.L, l = t % ti.L;
        T s = lds[k * ti.L + l];
        for (int w = 1; w < ti.nwaves; ++w) s += lds[(w * K + k) * ti.L + l];
        store(k, l, s);
    }
    __syncthreads();
}

static inline size_t lds_bytes(int waves, int L, int K) { return (size_t)waves * L * K * 8; }

}  // namespace fem
