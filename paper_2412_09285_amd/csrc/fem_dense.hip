// Dense-W MaxCut step for complete or near-complete graphs on gfx950 matrix
// cores.
//
// On a complete graph the field product phi = W m (m = tanh(h/2), the stored
// marginal copy, node-major [n][R]) is a dense matrix product n x n x R, so
// it runs on MFMA instead of the gather of the sparse kernel: a workgroup of
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

namespace fem {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int DK = 32;   // K block

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

    // epilogue: accumulator v of tile (bm, bn) is phi[row][r] with
    // row = 16 bm + kq + 4 v within the quarter, r = 16 bn + c16 (the
    // output layout of the f64 16x16x4 MFMA: lane group kq holds rows
    // kq, kq + 4, kq + 8, kq + 12 of column c16)
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
            const size_t sbase = (size_t)i * a.srow + r;
            float x, m1v, m2v;
            if constexpr (NT) {
                x = __builtin_nontemporal_load(a.h + sbase);
                m1v = __builtin_nontemporal_load(a.m1 + sbase);
                m2v = __builtin_nontemporal_load(a.m2 + sbase);
            } else {
                x = a.h[sbase];
                m1v = a.m1[sbase];
                m2v = a.m2[sbase];
            }
            const double phi = acc[bm][bn][v];
            const float ax = fabsf(x);
            const float e = expf(-ax);
            const float ope = 1.0f + e;
            const float pq = e / (ope * ope);   // P(1-P) without cancellation
            const float g = (float)((double)pq * (2.0 * phi + (double)x * sc.inv_beta_d));
            if constexpr (EN) {
                e_mphi[bn] += (double)tanhf(0.5f * x) * phi;
                e_h2[bn] += (double)(log1pf(e) + ax * (e / ope));
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
            const size_t base = (size_t)i * R + r;
            mn[base] = tanhf(0.5f * nh);
            if (a.grad) a.grad[base] = g;
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

hipError_t launch_dense_step(const Problem& p, int dtype, bool en, bool nt, int n_tiles, const StepArgs& a,
                             hipStream_t st)
{
    (void)hipGetLastError();   // drop stale errors of earlier calls
    if (!p.dense_w || p.kind != KIND_MAXCUT || dtype != 0 || p.dense_ld % DK != 0 || p.dense_ld % DENSE_ROWS != 0)
        return hipErrorInvalidValue;
    const dim3 g(n_tiles, (a.R + DENSE_COLS - 1) / DENSE_COLS), b(256);
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
