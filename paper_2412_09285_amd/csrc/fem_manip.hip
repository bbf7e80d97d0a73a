// Step kernels for the manipulated gradients (supplementary "The explicit
// gradient formulations" and "The explicit gradients and manipulated
// gradients for the benchmarking problems").
//
// The neighbours enter the manipulated gradient only through the one-hot
// vectors e_j of their current read-out, so the marginal copy that the
// gather reads shrinks to the read-out itself:
//   MaxCut: one bit per replica (1 = state (+), i.e. h > 0), rows of
//           ceil(R/32) 32-bit words, replica r in bit r % 32 of word r / 32;
//   bMinCut: one byte per (node, replica), the argmax state (ties to the
//           lowest state).
// A neighbour row is R/8 bytes (MaxCut) or R bytes (bMinCut) instead of
// 4 R q bytes of float32 marginals.
//
//   MaxCut:  g_i = gamma P_i (1 - P_i) [c_i sum_j W_ij s_j + h_i / beta],
//            s_j = +1 if h_j > 0 else -1, c_i = 1 / sum_j |W_ij|;
//   bMinCut: A(s) = -c^f_i sum_j W_ij e_j(s) + lam c^a_i [E~(s) - e_i(s)]
//                   + (h_i(s) - max h_i) / beta,
//            g_i(s) = gamma P_i(s) [A(s) - sum_s' P_i(s') A(s')],
//            c^f = q / sum_j W_ij, c^a = q / sqrt(sum_j W_ij), E~(s) the
//            centred count of nodes whose read-out is s.
// As in the explicit kernels, ln P + 1 is replaced by h - max h and the
// counts are centred: both differ by per-(node, replica) constants that the
// chain rule removes exactly.  A node without incident weight has c = 0.
// Per-replica energies are not formed: the manipulated gradient is not the
// gradient of the free energy being annealed.
#include "fem_device.h"

namespace fem {

// ======================================================== MaxCut (bits) ====
template <int V, bool NT>
__global__ void __launch_bounds__(step_max_threads(KIND_MAXCUT, V)) maxcut_manip_kernel(StepArgs a)
{
    const Tile tile = a.tiles[blk_tile(a.seg_major)];
    const int seg = blk_seg(a.seg_major);
    const TeamIdx ti = team_idx(a.lanes_log2);
    const int R = a.R;
    const int rb = (seg * ti.L + ti.tl) * V;
    const bool act = rb < R;
    const int word = rb >> 5, shift = rb & 31;
    // lanes whose replicas share one 32-bit word (within the team)
    const int G = (32 / V < ti.L) ? 32 / V : ti.L;
    const uint32_t* __restrict__ bc = static_cast<const uint32_t*>(a.marg_cur);
    uint32_t* __restrict__ bn = static_cast<uint32_t*>(a.marg_nxt);
    const StepScalars sc = a.sc;
    // every lane of a team walks the team's rows (the word assembly below
    // exchanges values inside the team); lanes past R only carry zeros
    for (int i = tile.row_begin + ti.team; i < tile.row_end; i += ti.teams) {
        uint32_t bits = 0;
        if (act) {
            const size_t base = (size_t)i * R + rb;
            const size_t sbase = (size_t)i * a.srow + rb;   // h, m1, m2 rows
            float hv[V], m1v[V], m2v[V], gv[V];
            ld_state<V, NT>(a.h + sbase, hv);
            ld_state<V, NT>(a.m1 + sbase, m1v);
            ld_state<V, NT>(a.m2 + sbase, m2v);
            double acc[V];
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] = 0.0;
            int64_t k = a.row_off[i];
            const int64_t kend = a.row_off[i + 1];
            for (; k + 4 <= kend; k += 4) {
                const int2 e0 = a.adj[k], e1 = a.adj[k + 1], e2 = a.adj[k + 2], e3 = a.adj[k + 3];
                const uint32_t b0 = bc[(size_t)e0.x * a.rw + word] >> shift;
                const uint32_t b1 = bc[(size_t)e1.x * a.rw + word] >> shift;
                const uint32_t b2 = bc[(size_t)e2.x * a.rw + word] >> shift;
                const uint32_t b3 = bc[(size_t)e3.x * a.rw + word] >> shift;
                const double w0 = __int_as_float(e0.y), w1 = __int_as_float(e1.y);
                const double w2 = __int_as_float(e2.y), w3 = __int_as_float(e3.y);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    acc[v] += ((b0 >> v) & 1u) ? w0 : -w0;
                    acc[v] += ((b1 >> v) & 1u) ? w1 : -w1;
                    acc[v] += ((b2 >> v) & 1u) ? w2 : -w2;
                    acc[v] += ((b3 >> v) & 1u) ? w3 : -w3;
                }
            }
            if (k + 2 <= kend) {   // a remaining pair in one round
                const int2 e0 = a.adj[k], e1 = a.adj[k + 1];
                const uint32_t b0 = bc[(size_t)e0.x * a.rw + word] >> shift;
                const uint32_t b1 = bc[(size_t)e1.x * a.rw + word] >> shift;
                const double w0 = __int_as_float(e0.y), w1 = __int_as_float(e1.y);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    acc[v] += ((b0 >> v) & 1u) ? w0 : -w0;
                    acc[v] += ((b1 >> v) & 1u) ? w1 : -w1;
                }
                k += 2;
            }
            if (k < kend) {
                const int2 e0 = a.adj[k];
                const uint32_t b0 = bc[(size_t)e0.x * a.rw + word] >> shift;
                const double w0 = __int_as_float(e0.y);
#pragma unroll
                for (int v = 0; v < V; ++v) acc[v] += ((b0 >> v) & 1u) ? w0 : -w0;
            }
            const double l1 = a.nrm[i];
            const double c = l1 > 0.0 ? 1.0 / l1 : 0.0;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const float x = hv[v];
                const float e = exp_neg(fabsf(x));
                const float r = rcp_f(1.0f + e);
                const float pq = e * r * r;         // P(1-P) without cancellation
                const float g = (float)(sc.gamma_d * ((double)pq * (c * acc[v] + (double)x * sc.inv_beta_d)));
                gv[v] = g;
                const float nh = adam_update(x, g, m1v[v], m2v[v], sc);
                hv[v] = nh;
                bits |= (nh > 0.0f ? 1u : 0u) << v;
            }
            st_state<V, NT>(a.h + sbase, hv);
            st_state<V, NT>(a.m1 + sbase, m1v);
            st_state<V, NT>(a.m2 + sbase, m2v);
            if (a.grad) st_f32<V>(a.grad + base, gv);
        }
        // assemble the word from the G lanes that share it (OR of disjoint
        // bit fields), written by the group's first lane
        uint32_t wv = bits << shift;
        for (int off = 1; off < G; off <<= 1) wv |= (uint32_t)__shfl_xor((int)wv, off, 64);
        if (act && (ti.tl & (G - 1)) == 0) bn[(size_t)i * a.rw + word] = wv;
    }
}

// sign bits of the fields: each half-wave forms one 32-bit word from 32
// coalesced loads and a ballot
__global__ void sign_bits_kernel(const float* __restrict__ h, int64_t srow, int32_t n, int32_t R, int32_t rw,
                                 uint32_t* __restrict__ out)
{
    const size_t words = (size_t)n * rw;
    const int lane = threadIdx.x & 63;
    const size_t wave = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const size_t nwaves = ((size_t)gridDim.x * blockDim.x) >> 6;
    for (size_t p = 2 * wave; p < words; p += 2 * nwaves) {
        const size_t k = p + (size_t)(lane >> 5);
        bool bit = false;
        if (k < words) {
            const size_t i = k / rw;
            const int r = 32 * (int)(k % rw) + (lane & 31);
            bit = r < R && h[i * srow + r] > 0.0f;
        }
        const uint64_t m = __ballot(bit);
        if (lane == 0) out[p] = (uint32_t)m;
        if (lane == 32 && p + 1 < words) out[p + 1] = (uint32_t)(m >> 32);
    }
}

// ===================================================== bMinCut (argmax) ====
template <int Q>
__device__ __forceinline__ int argmax_low(const float (&h)[Q])
{
    int b = 0;
#pragma unroll
    for (int s = 1; s < Q; ++s)
        if (h[s] > h[b]) b = s;
    return b;
}

template <int Q, bool NT>
__global__ void __launch_bounds__(step_max_threads(KIND_BMINCUT, Q)) potts_manip_kernel(StepArgs a)
{
    const Tile tile = a.tiles[blk_tile(a.seg_major)];
    const int seg = blk_seg(a.seg_major);
    const TeamIdx ti = team_idx(a.lanes_log2);
    const int R = a.R;
    const int r = seg * ti.L + ti.tl;
    const bool act = r < R;
    const uint8_t* __restrict__ ec = static_cast<const uint8_t*>(a.marg_cur);
    uint8_t* __restrict__ en = static_cast<uint8_t*>(a.marg_nxt);
    const StepScalars sc = a.sc;
    using AccT = typename std::conditional<(Q <= 8), double, float>::type;
    long long cs[Q];
#pragma unroll
    for (int s = 0; s < Q; ++s) cs[s] = 0;
    if (act) {
        double ct[Q];
#pragma unroll
        for (int s = 0; s < Q; ++s) ct[s] = a.ctil[((size_t)tile.inst * R + r) * Q + s];
        for (int i = tile.row_begin + ti.team; i < tile.row_end; i += ti.teams) {
            const size_t base = ((size_t)i * R + r) * Q;
            const size_t sbase = (size_t)i * a.srow + (size_t)r * Q;   // h, m1, m2 rows
            float hv[Q], m1v[Q], m2v[Q];
            ld_state<Q, NT>(a.h + sbase, hv);
            ld_state<Q, NT>(a.m1 + sbase, m1v);
            ld_state<Q, NT>(a.m2 + sbase, m2v);
            AccT phi[Q];
#pragma unroll
            for (int s = 0; s < Q; ++s) phi[s] = (AccT)0;
            int64_t k = a.row_off[i];
            const int64_t kend = a.row_off[i + 1];
            for (; k + 4 <= kend; k += 4) {
                const int2 e0 = a.adj[k], e1 = a.adj[k + 1], e2 = a.adj[k + 2], e3 = a.adj[k + 3];
                const int s0 = ec[(size_t)e0.x * R + r], s1 = ec[(size_t)e1.x * R + r];
                const int s2 = ec[(size_t)e2.x * R + r], s3 = ec[(size_t)e3.x * R + r];
                const AccT w0 = (AccT)__int_as_float(e0.y), w1 = (AccT)__int_as_float(e1.y);
                const AccT w2 = (AccT)__int_as_float(e2.y), w3 = (AccT)__int_as_float(e3.y);
#pragma unroll
                for (int s = 0; s < Q; ++s) {
                    phi[s] += (s0 == s) ? w0 : (AccT)0;
                    phi[s] += (s1 == s) ? w1 : (AccT)0;
                    phi[s] += (s2 == s) ? w2 : (AccT)0;
                    phi[s] += (s3 == s) ? w3 : (AccT)0;
                }
            }
            for (; k < kend; ++k) {
                const int2 e0 = a.adj[k];
                const int s0 = ec[(size_t)e0.x * R + r];
                const AccT w0 = (AccT)__int_as_float(e0.y);
#pragma unroll
                for (int s = 0; s < Q; ++s) phi[s] += (s0 == s) ? w0 : (AccT)0;
            }
            const int own = argmax_low<Q>(hv);
            // node weight: lam c^a V_i [sum_j V_j e_j(s) - V_i e_i(s)]; the
            // state counts become summed weights
            const int ivw = a.nw ? a.nw[i] : 1;
            const double vw = (double)ivw;
            const double D = a.nrm[i];
            const double cf = D > 0.0 ? (double)Q / D : 0.0;
            const double ca = D > 0.0 ? (double)Q / sqrt(D) : 0.0;
            float mx = hv[0];
#pragma unroll
            for (int s = 1; s < Q; ++s) mx = fmaxf(mx, hv[s]);
            float P[Q], Z = 0.0f;
#pragma unroll
            for (int s = 0; s < Q; ++s) { P[s] = exp_neg(mx - hv[s]); Z += P[s]; }
            const float invZ = rcp_f(Z);
#pragma unroll
            for (int s = 0; s < Q; ++s) P[s] *= invZ;
            // mean normalised by the sum of the float32 marginals (their
            // rounding then perturbs only the weights)
            auto Aof = [&](int s) {
                return -cf * (double)phi[s] + sc.lam_d * ca * vw * (ct[s] - (own == s ? vw : 0.0)) +
                       ((double)hv[s] - (double)mx) * sc.inv_beta_d;
            };
            double avg = 0.0, psum = 0.0;
#pragma unroll
            for (int s = 0; s < Q; ++s) {
                avg = fma((double)P[s], Aof(s), avg);
                psum += (double)P[s];
            }
            avg /= psum;
            float gv[Q];
#pragma unroll
            for (int s = 0; s < Q; ++s) gv[s] = (float)(sc.gamma_d * ((Aof(s) - avg) * (double)P[s]));
#pragma unroll
            for (int s = 0; s < Q; ++s) hv[s] = adam_update(hv[s], gv[s], m1v[s], m2v[s], sc);
            const int nw = argmax_low<Q>(hv);
#pragma unroll
            for (int s = 0; s < Q; ++s) cs[s] += (nw == s) ? ivw : 0;
            st_state<Q, NT>(a.h + sbase, hv);
            st_state<Q, NT>(a.m1 + sbase, m1v);
            st_state<Q, NT>(a.m2 + sbase, m2v);
            en[(size_t)i * R + r] = (uint8_t)nw;
            if (a.grad) st_f32<Q>(a.grad + base, gv);
        }
    }
    extern __shared__ double lds_d[];
    block_reduce_store<long long, Q>(cs, ti, a.lanes_log2, reinterpret_cast<long long*>(lds_d),
                                     [&](int s, int l, long long v) {
                                         const int rr = seg * ti.L + l;
                                         if (rr < R) a.cpart[((size_t)tile.slot * R + rr) * Q + s] = v;
                                     });
}

// read-out of the fields and its per-tile state counts
template <int Q>
__global__ void __launch_bounds__(step_max_threads(KIND_BMINCUT, Q)) potts_manip_init_kernel(StepArgs a)
{
    const Tile tile = a.tiles[blk_tile(a.seg_major)];
    const int seg = blk_seg(a.seg_major);
    const TeamIdx ti = team_idx(a.lanes_log2);
    const int R = a.R;
    const int r = seg * ti.L + ti.tl;
    uint8_t* __restrict__ en = static_cast<uint8_t*>(a.marg_nxt);
    long long cs[Q];
#pragma unroll
    for (int s = 0; s < Q; ++s) cs[s] = 0;
    if (r < R) {
        for (int i = tile.row_begin + ti.team; i < tile.row_end; i += ti.teams) {
            float hv[Q];
            ld_f32<Q>(a.h + (size_t)i * a.srow + (size_t)r * Q, hv);
            const int b = argmax_low<Q>(hv);
#pragma unroll
            for (int s = 0; s < Q; ++s) cs[s] += (b == s) ? (a.nw ? a.nw[i] : 1) : 0;
            en[(size_t)i * R + r] = (uint8_t)b;
        }
    }
    extern __shared__ double lds_d[];
    block_reduce_store<long long, Q>(cs, ti, a.lanes_log2, reinterpret_cast<long long*>(lds_d),
                                     [&](int s, int l, long long v) {
                                         const int rr = seg * ti.L + l;
                                         if (rr < R) a.cpart[((size_t)tile.slot * R + rr) * Q + s] = v;
                                     });
}

// ================================================================ launch ===
template <bool NT>
static hipError_t launch_manip_t(int kind, int vec, const LaunchGeom& geo, int waves, const StepArgs& a,
                                 hipStream_t st)
{
    const dim3 g = geo.seg_major ? dim3(geo.nseg, geo.n_tiles) : dim3(geo.n_tiles, geo.nseg);
    const dim3 b(64 * waves);
    if (kind == KIND_MAXCUT) {
        switch (vec) {
        case 1: maxcut_manip_kernel<1, NT><<<g, b, 0, st>>>(a); break;
        case 2: maxcut_manip_kernel<2, NT><<<g, b, 0, st>>>(a); break;
        case 4: maxcut_manip_kernel<4, NT><<<g, b, 0, st>>>(a); break;
        case 8: maxcut_manip_kernel<8, NT><<<g, b, 0, st>>>(a); break;
        default: return hipErrorInvalidValue;
        }
    } else if (kind == KIND_BMINCUT) {
        const size_t lds = lds_bytes(waves, geo.lanes, a.q);
        switch (a.q) {
        case 2: potts_manip_kernel<2, NT><<<g, b, lds, st>>>(a); break;
        case 4: potts_manip_kernel<4, NT><<<g, b, lds, st>>>(a); break;
        case 8: potts_manip_kernel<8, NT><<<g, b, lds, st>>>(a); break;
        case 16: potts_manip_kernel<16, NT><<<g, b, lds, st>>>(a); break;
        case 32: potts_manip_kernel<32, NT><<<g, b, lds, st>>>(a); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_manip_step(int kind, int vec, bool nt, const LaunchGeom& g, int waves, const StepArgs& a,
                             hipStream_t st)
{
    (void)hipGetLastError();   // drop stale errors of earlier calls
    return nt ? launch_manip_t<true>(kind, vec, g, waves, a, st) : launch_manip_t<false>(kind, vec, g, waves, a, st);
}

hipError_t launch_manip_init(int kind, const LaunchGeom& geo, int waves, const StepArgs& a, hipStream_t st)
{
    (void)hipGetLastError();   // drop stale errors of earlier calls
    if (kind == KIND_MAXCUT) {
        const size_t count = (size_t)a.n * a.rw;   // words, two per wave
        if (count == 0) return hipSuccess;
        const size_t blocks = (count + 7) / 8;
        sign_bits_kernel<<<(unsigned)(blocks < 65536 ? blocks : 65536), 256, 0, st>>>(
            a.h, a.srow, a.n, a.R, a.rw, static_cast<uint32_t*>(a.marg_nxt));
        return hipGetLastError();
    }
    if (kind != KIND_BMINCUT) return hipErrorInvalidValue;
    const dim3 g = geo.seg_major ? dim3(geo.nseg, geo.n_tiles) : dim3(geo.n_tiles, geo.nseg);
    const dim3 b(64 * waves);
    const size_t lds = lds_bytes(waves, geo.lanes, a.q);
    switch (a.q) {
    case 2: potts_manip_init_kernel<2><<<g, b, lds, st>>>(a); break;
    case 4: potts_manip_init_kernel<4><<<g, b, lds, st>>>(a); break;
    case 8: potts_manip_init_kernel<8><<<g, b, lds, st>>>(a); break;
    case 16: potts_manip_init_kernel<16><<<g, b, lds, st>>>(a); break;
    case 32: potts_manip_init_kernel<32><<<g, b, lds, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fem
