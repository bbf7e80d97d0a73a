// Dense-W MaxCut step for complete or near-complete graphs on gfx950 matrix
// cores.
//
// On a complete graph the field product phi = W m (m = tanh(h/2)) is a dense
// matrix product n x n x R, so it runs on MFMA instead of the gather of the
// sparse kernel.  Two kernels, both as exact as the sparse kernel's FP64
// accumulation: for integral weights (|W| <= 127) int8 products of the
// fixed-point marginals' digit planes (maxcut_dense_i8_step_kernel, second
// half of this file); for any other W the FP64 kernel below.
//
// FP64 kernel: the marginal copy is float, node-major [n][R]; a workgroup of
// four waves owns a 64-row x 64-replica block of phi, each wave a 32 x 32
// quarter held as 2 x 2 tiles of v_mfma_f64_16x16x4_f64 accumulators.  The
// products and sums are formed in double, as the sparse kernel accumulates:
// near equilibrium the gradient 2 phi + h / beta is a small difference, and
// float32 accumulation over ~10^3 neighbours leaves errors of order 1e-5 of
// the gradient there (a float32 matrix-core variant measured 1.0e-5 on a
// 300-node complete graph).  K (the neighbour index j) advances in blocks
// of 32 through double-buffered LDS (float; widened when fed to the MFMA):
// the A block is read from rows j of W (W is symmetric, so row j holds
// column j: both operands are staged from contiguous rows, no transpose), the
// B block from rows j of the marginal copy; global loads of block k+1 are in
// flight while the MFMAs consume block k.
//
// The epilogue is the explicit-gradient MaxCut step of the sparse kernel
// (one-logit reduction, supplementary "Simplification of FEM for solving the
// MaxCut problem"): g_i = P_i (1 - P_i) [2 phi_i + h_i / beta], the optimiser
// update, the new marginal, and per-replica energy partials [sum m phi,
// sum H2(P)] for the tile's rows; the gradient terms are combined in double
// as there.
#include "fem_device.h"
#include "fem_dense.h"

#include <algorithm>

namespace fem {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

constexpr int DK = 32;   // K block of the FP64 kernel

// h, m1, m2 of (node i, replica r).  The kernels load every entry of the
// lane before the K loop, so that these loads are in flight while the
// matrix cores run (issued after the first store they would wait for it:
// the state arrays may alias as far as the compiler knows).
template <bool NT>
__device__ __forceinline__ void dense_load(const StepArgs& a, int i, int r, float& x, float& m1v, float& m2v)
{
    const size_t sbase = (size_t)i * a.srow + r;
    if constexpr (NT) {
        x = __builtin_nontemporal_load(a.h + sbase);
        m1v = __builtin_nontemporal_load(a.m1 + sbase);
        m2v = __builtin_nontemporal_load(a.m2 + sbase);
    } else {
        x = a.h[sbase];
        m1v = a.m1[sbase];
        m2v = a.m2[sbase];
    }
}

// The step of one (node i, replica r) given its field phi and loaded state:
// gradient, the optimiser update of h, m1, m2, energy terms; returns the new
// marginal and stores the gradient when it is kept.
template <bool EN, bool NT>
__device__ __forceinline__ float dense_update(const StepArgs& a, const StepScalars& sc, int i, int r, double phi,
                                              float x, float m1v, float m2v, double& e_mphi, double& e_h2)
{
    const size_t sbase = (size_t)i * a.srow + r;
    const float ax = fabsf(x);
    const float e = exp_neg(ax);
    const float rr = rcp_f(1.0f + e);
    const float pmin = e * rr;          // min(P, 1 - P)
    const float pq = pmin * rr;         // P(1-P) without cancellation
    const float g = (float)((double)pq * fma((double)x, sc.inv_beta_d, 2.0 * phi));
    if constexpr (EN) {
        // own marginal sign(h) (1 - e) / (1 + e): its cancellation near h = 0
        // leaves an absolute error of about 1e-7, far below the scale of U
        e_mphi += (double)copysignf((1.0f - e) * rr, x) * phi;
        e_h2 += (double)(log1p_f(e) + ax * pmin);
    }
    const float nh = adam_update(x, g, m1v, m2v, sc);
    if constexpr (NT) {
        __builtin_nontemporal_store(nh, a.h + sbase);
        __builtin_nontemporal_store(m1v, a.m1 + sbase);
        __builtin_nontemporal_store(m2v, a.m2 + sbase);
    } else {
        a.h[sbase] = nh;
        a.m1[sbase] = m1v;
        a.m2[sbase] = m2v;
    }
    if (a.grad) a.grad[(size_t)i * a.R + r] = g;
    return tanh_half(nh);
}

template <bool EN, bool NT>
__global__ void __launch_bounds__(256) maxcut_dense_step_kernel(StepArgs a, const float* __restrict__ W, int32_t ld)
{
    constexpr int DM = DENSE_ROWS, DN = DENSE_COLS;
    const Tile tile = a.tiles[blockIdx.x];
    const int i0 = tile.row_begin;   // a multiple of DM
    const int r0 = blockIdx.y * DN;
    const int R = a.R, n = a.n;
    const float* __restrict__ mc = static_cast<const float*>(a.marg_cur);
    float* __restrict__ mn = static_cast<float*>(a.marg_nxt);
    __shared__ float sA[2][DK][DM];   // sA[.][k][m] = W[j0 + k][i0 + m]
    __shared__ float sB[2][DK][DN];   // sB[.][k][c] = m[j0 + k][r0 + c]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;   // the wave's 32 x 32 quarter
    const int kq = lane >> 4, c16 = lane & 15;   // MFMA lane: k index, row / column
    // staging: thread (wave, lane) moves column `lane` of K rows wave + 4u
    const bool bcol = r0 + lane < R;
    float ra[DK / 4], rb[DK / 4];
    auto gload = [&](int j0) {
#pragma unroll
        for (int u = 0; u < DK / 4; ++u) {
            const int j = j0 + wave + 4 * u;   // < ld: W is zero-padded to ld rows and columns
            ra[u] = W[(size_t)j * ld + i0 + lane];
            rb[u] = (j < n && bcol) ? mc[(size_t)j * R + r0 + lane] : 0.0f;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int u = 0; u < DK / 4; ++u) {
            sA[buf][wave + 4 * u][lane] = ra[u];
            sB[buf][wave + 4 * u][lane] = rb[u];
        }
    };
    // this lane's 16 outputs: tile (bm, bn), register v -> row
    // 16 bm + kq + 4 v of the quarter, replica 16 bn + c16 (the output layout
    // of the f64 16x16x4 MFMA: lane group kq holds rows kq, kq + 4, kq + 8,
    // kq + 12 of column c16); their state is loaded up front
    float xs[2][8], m1s[2][8], m2s[2][8];
#pragma unroll
    for (int bn = 0; bn < 2; ++bn) {
        const int r = r0 + wn * 32 + 16 * bn + c16;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i = i0 + wm * 32 + 16 * (q >> 2) + kq + 4 * (q & 3);
            xs[bn][q] = m1s[bn][q] = m2s[bn][q] = 0.0f;
            if (r < R && i < tile.row_end) dense_load<NT>(a, i, r, xs[bn][q], m1s[bn][q], m2s[bn][q]);
        }
    }
    f64x4 acc[2][2];   // [16-row tile][16-column tile]
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
        for (int bn = 0; bn < 2; ++bn)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[bm][bn][v] = 0.0;
    const int nk = ld / DK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kb = 0; kb < nk; ++kb) {
        const int buf = kb & 1;
        if (kb + 1 < nk) gload((kb + 1) * DK);
#pragma unroll
        for (int kk = 0; kk < DK / 4; ++kk) {
            // A(lane) = A[m = c16][k = 4 kk + kq], B(lane) = B[k = 4 kk + kq][n = c16]
            const int k = 4 * kk + kq;
            double av[2], bv[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                av[t] = (double)sA[buf][k][wm * 32 + 16 * t + c16];
                bv[t] = (double)sB[buf][k][wn * 32 + 16 * t + c16];
            }
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                for (int bn = 0; bn < 2; ++bn)
                    acc[bm][bn] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bm], bv[bn], acc[bm][bn], 0, 0, 0);
        }
        // buffer buf ^ 1 was last read before the previous barrier
        if (kb + 1 < nk) sstore(buf ^ 1);
        __syncthreads();
    }

    // epilogue
    const StepScalars sc = a.sc;
    double e_mphi[2] = {0.0, 0.0}, e_h2[2] = {0.0, 0.0};
#pragma unroll
    for (int bn = 0; bn < 2; ++bn) {
        const int r = r0 + wn * 32 + 16 * bn + c16;
        if (r >= R) continue;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int bm = q >> 2, v = q & 3;
            const int i = i0 + wm * 32 + 16 * bm + kq + 4 * v;
            if (i >= tile.row_end) continue;
            mn[(size_t)i * R + r] = dense_update<EN, NT>(a, sc, i, r, acc[bm][bn][v], xs[bn][q], m1s[bn][q],
                                                         m2s[bn][q], e_mphi[bn], e_h2[bn]);
        }
    }
    if constexpr (EN) {
        // the four lane groups kq hold the same replicas (butterfly); then the
        // two waves of a column pair (wm = 0, 1) in order
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) {
            e_mphi[bn] += __shfl_xor(e_mphi[bn], 16, 64);
            e_h2[bn] += __shfl_xor(e_h2[bn], 16, 64);
            e_mphi[bn] += __shfl_xor(e_mphi[bn], 32, 64);
            e_h2[bn] += __shfl_xor(e_h2[bn], 32, 64);
        }
        __shared__ double sE[2][2][2][16];   // [wn][bn][term][c16], from wm = 1
        if (wm == 1 && kq == 0) {
#pragma unroll
            for (int bn = 0; bn < 2; ++bn) {
                sE[wn][bn][0][c16] = e_mphi[bn];
                sE[wn][bn][1][c16] = e_h2[bn];
            }
        }
        __syncthreads();
        if (wm == 0 && kq == 0) {
#pragma unroll
            for (int bn = 0; bn < 2; ++bn) {
                const int r = r0 + wn * 32 + 16 * bn + c16;
                if (r < R) {
                    a.epart[((size_t)tile.slot * 2 + 0) * R + r] = e_mphi[bn] + sE[wn][bn][0][c16];
                    a.epart[((size_t)tile.slot * 2 + 1) * R + r] = e_h2[bn] + sE[wn][bn][1][c16];
                }
            }
        }
    }
}

// ------------------------------------------------ integer weights: int8 ---
// For integral W with |W_ij| <= 127 the marginal copy is kept in fixed point,
// m_fx = rint(m 2^30) (|m| <= 1, so |m_fx| <= 2^30), written as four signed
// base-256 digits m_fx = d0 + 2^8 d1 + 2^16 d2 + 2^24 d3 (d0..d2 in
// [-128, 127], |d3| <= 65).  Each digit plane is an int8 matrix, and
// S_d = W d_d is an exact int32 product on the int8 matrix cores
// (v_mfma_i32_32x32x32_i8; |S_d| <= 127 * 128 * n < 2^31 for n <= 32768), so
// phi = 2^-30 sum_d 2^(8d) S_d is the field of the fixed-point marginals
// without any rounding (all terms are integers below 2^53).  Against the
// float32 copy the only difference is the quantisation of m to 2^-30.
// Planes are replica-major, q[d][r][j] with rows of ld bytes and Rp (R
// rounded up to 64) rows per plane, so that an MFMA lane's 16 consecutive k
// values are 16 contiguous bytes of one row; rows j >= n and replicas r >= R
// hold zeros.
constexpr int QK = DENSE_LD_ALIGN;   // K block (bytes of a row per block)
constexpr int QP = QK + 16;          // LDS row pitch: 16-byte reads of 32 rows stay conflict-free

__device__ __forceinline__ void to_digits(float m, int (&d)[4])
{
    int x = (int)rintf(m * 1073741824.0f);   // exact scaling by 2^30
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        d[k] = ((x & 0xff) ^ 0x80) - 0x80;   // low byte as a signed digit
        x = (x - d[k]) >> 8;                  // exact: x - d[k] is a multiple of 256
    }
    d[3] = x;
}

template <bool EN, bool NT>
__global__ void __launch_bounds__(256) maxcut_dense_i8_step_kernel(StepArgs a, const int8_t* __restrict__ W8,
                                                                   int32_t ld, int32_t Rp)
{
    constexpr int DM = DENSE_ROWS, DN = DENSE_COLS;
    const Tile tile = a.tiles[blockIdx.x];
    const int i0 = tile.row_begin;   // a multiple of DM
    const int r0 = blockIdx.y * DN;
    const int R = a.R;
    const size_t plane = (size_t)Rp * ld;
    const int8_t* __restrict__ qc = static_cast<const int8_t*>(a.marg_cur);
    int8_t* __restrict__ qn = static_cast<int8_t*>(a.marg_nxt);
    __shared__ __attribute__((aligned(16))) int8_t sA[DM][QP];      // W[i0 + m][j0 + k]
    __shared__ __attribute__((aligned(16))) int8_t sB[4][DN][QP];   // q[d][r0 + c][j0 + k]
    __shared__ double sE[2][2][32];                                    // energy partials of waves wm = 1
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;   // the wave's 32 x 32 quarter
    const int kh = lane >> 5, c32 = lane & 31;
    // staging: 16-byte chunks ck = t + 256 c; chunk ck is piece ck % 8 of row
    // ck / 8 of the W block (2 per thread), and of row (ck / 8) % 64 of digit
    // plane ck / 512 (8 per thread).  One LDS buffer: the next block's loads
    // are in registers while the MFMAs read the current one (a second buffer
    // at half the block measured slower).
    i32x4 ra[2], rb[8];
    auto gload = [&](int j0) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int ck = tid + 256 * c, row = ck >> 3, ch = (ck & 7) * 16;
            ra[c] = *reinterpret_cast<const i32x4*>(W8 + (size_t)(i0 + row) * ld + j0 + ch);
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int ck = tid + 256 * c, d = ck >> 9, row = (ck >> 3) & 63, ch = (ck & 7) * 16;
            rb[c] = *reinterpret_cast<const i32x4*>(qc + d * plane + (size_t)(r0 + row) * ld + j0 + ch);
        }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int ck = tid + 256 * c, row = ck >> 3, ch = (ck & 7) * 16;
            *reinterpret_cast<i32x4*>(&sA[row][ch]) = ra[c];
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int ck = tid + 256 * c, d = ck >> 9, row = (ck >> 3) & 63, ch = (ck & 7) * 16;
            *reinterpret_cast<i32x4*>(&sB[d][row][ch]) = rb[c];
        }
    };
    // this lane's 16 outputs: register v -> row 8 (v / 4) + 4 kh + v % 4 of
    // the quarter, replica c32; their state is loaded up front
    const int r = r0 + wn * 32 + c32;
    float xs[16], m1s[16], m2s[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int i = i0 + wm * 32 + 8 * (v >> 2) + 4 * kh + (v & 3);
        xs[v] = m1s[v] = m2s[v] = 0.0f;
        if (r < R && i < tile.row_end) dense_load<NT>(a, i, r, xs[v], m1s[v], m2s[v]);
    }
    i32x16 acc[4];
#pragma unroll
    for (int d = 0; d < 4; ++d)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[d][v] = 0;
    const int nk = ld / QK;
    gload(0);
    for (int kb = 0; kb < nk; ++kb) {
        sstore();
        __syncthreads();
        if (kb + 1 < nk) gload((kb + 1) * QK);
#pragma unroll
        for (int kk = 0; kk < QK / 32; ++kk) {
            // lane (kh, c32) supplies k = 32 kk + 16 kh + e, e = 0..15, of row
            // c32 of A and of column c32 of B (the same pairing on both sides)
            const i32x4 av = *reinterpret_cast<const i32x4*>(&sA[wm * 32 + c32][32 * kk + 16 * kh]);
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const i32x4 bv = *reinterpret_cast<const i32x4*>(&sB[d][wn * 32 + c32][32 * kk + 16 * kh]);
                acc[d] = __builtin_amdgcn_mfma_i32_32x32x32_i8(av, bv, acc[d], 0, 0, 0);
            }
        }
        __syncthreads();
    }

    // epilogue: new marginals go to LDS as digits, transposed to
    // [d][replica][row], then out as 64-byte rows
    int8_t (*sT)[DN][QP] = sB;   // [4][DN][QP]: the staging buffer, free after the K loop
    const StepScalars sc = a.sc;
    double e_mphi = 0.0, e_h2 = 0.0;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int il = wm * 32 + 8 * (v >> 2) + 4 * kh + (v & 3);
        const int i = i0 + il;
        float mnew = 0.0f;   // rows past n and replicas past R keep zero digits
        if (r < R && i < tile.row_end) {
            const double phi = ((double)acc[3][v] * 16777216.0 + (double)acc[2][v] * 65536.0 +
                                (double)acc[1][v] * 256.0 + (double)acc[0][v]) * (1.0 / 1073741824.0);
            mnew = dense_update<EN, NT>(a, sc, i, r, phi, xs[v], m1s[v], m2s[v], e_mphi, e_h2);
        }
        int dg[4];
        to_digits(mnew, dg);
#pragma unroll
        for (int d = 0; d < 4; ++d) sT[d][wn * 32 + c32][il] = (int8_t)dg[d];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int c = tid + 256 * u;   // chunk: plane d, replica row rl, 16-byte piece
        const int d = c >> 8, rl = (c >> 2) & 63, ch = (c & 3) * 16;
        if (r0 + rl < R)
            *reinterpret_cast<i32x4*>(qn + d * plane + (size_t)(r0 + rl) * ld + i0 + ch) =
                *reinterpret_cast<const i32x4*>(&sT[d][rl][ch]);
    }
    if constexpr (EN) {
        e_mphi += __shfl_xor(e_mphi, 32, 64);
        e_h2 += __shfl_xor(e_h2, 32, 64);
        if (wm == 1 && kh == 0) {
            sE[wn][0][c32] = e_mphi;
            sE[wn][1][c32] = e_h2;
        }
        __syncthreads();
        if (wm == 0 && kh == 0 && r < R) {
            a.epart[((size_t)tile.slot * 2 + 0) * R + r] = e_mphi + sE[wn][0][c32];
            a.epart[((size_t)tile.slot * 2 + 1) * R + r] = e_h2 + sE[wn][1][c32];
        }
    }
}

// digit planes of the marginals of h (rows j < n, replicas r < R)
__global__ void dense_i8_init_kernel(const float* __restrict__ h, int64_t srow, int32_t n, int32_t R, int32_t ld,
                                     size_t plane, int8_t* __restrict__ q)
{
    const size_t total = (size_t)n * R;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(k / n), j = (int)(k % n);
        int dg[4];
        to_digits(tanh_half(h[(size_t)j * srow + r]), dg);
#pragma unroll
        for (int d = 0; d < 4; ++d) q[d * plane + (size_t)r * ld + j] = (int8_t)dg[d];
    }
}

hipError_t launch_dense_i8_init(const Problem& p, const StepArgs& a, hipStream_t st)
{
    (void)hipGetLastError();   // drop stale errors of earlier calls
    if (!p.dense_w8 || p.dense_ld % QK != 0) return hipErrorInvalidValue;
    const int Rp = dense_rows_padded(a.R);
    const size_t total = (size_t)a.n * a.R;
    const size_t blocks = std::min<size_t>((total + 255) / 256, 65536);
    dense_i8_init_kernel<<<(unsigned)std::max<size_t>(blocks, 1), 256, 0, st>>>(
        a.h, a.srow, a.n, a.R, p.dense_ld, (size_t)Rp * p.dense_ld, static_cast<int8_t*>(a.marg_nxt));
    return hipGetLastError();
}

hipError_t launch_dense_step(const Problem& p, int dtype, bool en, bool nt, int n_tiles, const StepArgs& a,
                             hipStream_t st)
{
    (void)hipGetLastError();   // drop stale errors of earlier calls
    if (!p.dense_w || p.kind != KIND_MAXCUT || dtype != 0 || p.dense_ld % QK != 0 || p.dense_ld % DENSE_ROWS != 0)
        return hipErrorInvalidValue;
    const dim3 g(n_tiles, (a.R + DENSE_COLS - 1) / DENSE_COLS), b(256);
    if (p.dense_w8) {
        const int Rp = dense_rows_padded(a.R);
        if (en) {
            if (nt) maxcut_dense_i8_step_kernel<true, true><<<g, b, 0, st>>>(a, p.dense_w8, p.dense_ld, Rp);
            else maxcut_dense_i8_step_kernel<true, false><<<g, b, 0, st>>>(a, p.dense_w8, p.dense_ld, Rp);
        } else {
            if (nt) maxcut_dense_i8_step_kernel<false, true><<<g, b, 0, st>>>(a, p.dense_w8, p.dense_ld, Rp);
            else maxcut_dense_i8_step_kernel<false, false><<<g, b, 0, st>>>(a, p.dense_w8, p.dense_ld, Rp);
        }
        return hipGetLastError();
    }
    if (en) {
        if (nt) maxcut_dense_step_kernel<true, true><<<g, b, 0, st>>>(a, p.dense_w, p.dense_ld);
        else maxcut_dense_step_kernel<true, false><<<g, b, 0, st>>>(a, p.dense_w, p.dense_ld);
    } else {
        if (nt) maxcut_dense_step_kernel<false, true><<<g, b, 0, st>>>(a, p.dense_w, p.dense_ld);
        else maxcut_dense_step_kernel<false, false><<<g, b, 0, st>>>(a, p.dense_w, p.dense_ld);
    }
    return hipGetLastError();
}

}  // namespace fem
