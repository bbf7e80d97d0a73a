// HIP kernels of the FEM hot path for gfx950 (CDNA4, wave64).
//
// One step kernel per problem kind fuses, for a tile of rows (nodes or
// variables) and all replicas:
//   gather of neighbour marginals (sparse product W . m, W . P, or the
//   clause cavity products) -> gradient dF/dh -> Adam -> new marginal copy,
// plus optional per-replica energy partials.  The gradient formulas are the
// paper's explicit gradients (supplementary "The explicit gradients and
// manipulated gradients ...", with the discretisation and normalisers of the
// manipulated variant left out, i.e. c_i = 1, e_j -> P_j, gamma_grad = 1)
// pushed through the softmax chain rule ("The explicit gradient formulations"),
// and for q = 2 the one-logit reduction ("Simplification of FEM for solving the
// MaxCut problem").
//
// Layout: rows are node-major with the replica index fastest (then the Potts
// state), so one neighbour gather reads R*q contiguous values.  A "team" of L
// lanes (L a power of two <= 64) owns one row at a time; lane l holds V
// consecutive replicas (one-logit kinds) or one replica's q states (Potts).
// Several teams share a wave when L < 64.  A workgroup owns one tile, a row
// range of a single instance, so per-instance reductions never mix instances.
//
// Determinism: every sum has a fixed order (CSR order for gathers, butterfly
// then wave order inside a workgroup, tile order across workgroups).  The
// Potts column sums, which feed back into the gradient, are accumulated in
// 2^-40 fixed point (int64), so they do not depend on the tile shape at all.
#include "fem_device.h"

#include <type_traits>

namespace fem {

// Adjacency entry k as {column, float bits of the weight}; with PM1 (every
// weight +-1) from the 4-byte form, the sign in bit 31 of the column.
template <bool PM1>
__device__ __forceinline__ int2 ld_adj(const StepArgs& a, int64_t k)
{
    if constexpr (PM1) {
        const uint32_t e = (uint32_t)a.adj_pm1[k];
        return make_int2((int)(e & 0x7fffffffu), (int)(0x3f800000u | (e & 0x80000000u)));
    } else {
        return a.adj[k];
    }
}

// ========================================================= MaxCut step ====
// phi_i = sum_j W_ij m_j with m = tanh(h/2) = 2P - 1 (the stored copy);
// g_i = P_i (1 - P_i) [2 phi_i + h_i / beta]: the explicit gradient of the
// ordered-pair F through the one-logit reduction.  Energies: U = -W_tot +
// (1/2) sum_i m_i phi_i and S = sum_i H2(P_i), accumulated here as
// [sum m phi, sum H2] per replica.
template <int V, typename MT, bool EN, bool NT, bool PM1>
__global__ void __launch_bounds__(step_max_threads(KIND_MAXCUT, V)) maxcut_step_kernel(StepArgs a)
{
    const Tile tile = a.tiles[blk_tile(a.seg_major)];
    const int seg = blk_seg(a.seg_major);
    const TeamIdx ti = team_idx(a.lanes_log2);
    const int R = a.R;
    const int rb = (seg * ti.L + ti.tl) * V;
    const bool act = rb < R;
    const MT* __restrict__ mc = static_cast<const MT*>(a.marg_cur);
    MT* __restrict__ mn = static_cast<MT*>(a.marg_nxt);
    const StepScalars sc = a.sc;
    // the field sums and the gradient combination are formed in double for
    // either marginal type: near equilibrium g is a small difference of
    // 2 phi and h / beta, and float sums of neighbour values that span many
    // binades would lose the low bits of that difference
    using CT = double;
    // per-lane energy terms over the few rows of one team (float), widened
    // to double for the workgroup and tile sums
    float eacc[2 * V];
#pragma unroll
    for (int k = 0; k < 2 * V; ++k) eacc[k] = 0.0f;

    if (act) {
        for (int i = tile.row_begin + ti.team; i < tile.row_end; i += ti.teams) {
            // the row's own state first: its loads overlap the neighbour gather
            const size_t base = (size_t)i * R + rb;
            const size_t sbase = (size_t)i * a.srow + rb;   // h, m1, m2 rows
            float hv[V], m1v[V], m2v[V], mnew[V], gv[V];
            ld_state<V, NT>(a.h + sbase, hv);
            ld_state<V, NT>(a.m1 + sbase, m1v);
            ld_state<V, NT>(a.m2 + sbase, m2v);
            CT acc[V];
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] = (CT)0;
            int64_t k = a.row_off[i];
            const int64_t kend = a.row_off[i + 1];
            if constexpr (V == 1) {
                // one value per lane (few replicas, dense rows): rounds of
                // sixteen, then eight neighbours in flight shorten the row's
                // latency chain
                for (; k + 16 <= kend; k += 16) {
                    int2 e[16];
                    float x[16][1];
#pragma unroll
                    for (int u = 0; u < 16; ++u) e[u] = ld_adj<PM1>(a, k + u);
#pragma unroll
                    for (int u = 0; u < 16; ++u) ld_marg<MT, 1>(mc + (size_t)e[u].x * R + rb, x[u]);
#pragma unroll
                    for (int u = 0; u < 16; ++u) acc[0] = fma((CT)__int_as_float(e[u].y), (CT)x[u][0], acc[0]);
                }
                for (; k + 8 <= kend; k += 8) {
                    int2 e[8];
                    float x[8][1];
#pragma unroll
                    for (int u = 0; u < 8; ++u) e[u] = ld_adj<PM1>(a, k + u);
#pragma unroll
                    for (int u = 0; u < 8; ++u) ld_marg<MT, 1>(mc + (size_t)e[u].x * R + rb, x[u]);
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc[0] = fma((CT)__int_as_float(e[u].y), (CT)x[u][0], acc[0]);
                }
            }
            for (; k + 4 <= kend; k += 4) {
                const int2 e0 = ld_adj<PM1>(a, k), e1 = ld_adj<PM1>(a, k + 1), e2 = ld_adj<PM1>(a, k + 2), e3 = ld_adj<PM1>(a, k + 3);
                float x0[V], x1[V], x2[V], x3[V];
                ld_marg<MT, V>(mc + (size_t)e0.x * R + rb, x0);
                ld_marg<MT, V>(mc + (size_t)e1.x * R + rb, x1);
                ld_marg<MT, V>(mc + (size_t)e2.x * R + rb, x2);
                ld_marg<MT, V>(mc + (size_t)e3.x * R + rb, x3);
                const CT w0 = __int_as_float(e0.y), w1 = __int_as_float(e1.y);
                const CT w2 = __int_as_float(e2.y), w3 = __int_as_float(e3.y);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    acc[v] = fma(w0, (CT)x0[v], acc[v]);
                    acc[v] = fma(w1, (CT)x1[v], acc[v]);
                    acc[v] = fma(w2, (CT)x2[v], acc[v]);
                    acc[v] = fma(w3, (CT)x3[v], acc[v]);
                }
            }
            if (k + 2 <= kend) {   // a remaining pair in one round
                const int2 e0 = ld_adj<PM1>(a, k), e1 = ld_adj<PM1>(a, k + 1);
                float x0[V], x1[V];
                ld_marg<MT, V>(mc + (size_t)e0.x * R + rb, x0);
                ld_marg<MT, V>(mc + (size_t)e1.x * R + rb, x1);
                const CT w0 = __int_as_float(e0.y), w1 = __int_as_float(e1.y);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    acc[v] = fma(w0, (CT)x0[v], acc[v]);
                    acc[v] = fma(w1, (CT)x1[v], acc[v]);
                }
                k += 2;
            }
            if (k < kend) {
                const int2 e0 = ld_adj<PM1>(a, k);
                float x0[V];
                ld_marg<MT, V>(mc + (size_t)e0.x * R + rb, x0);
                const CT w0 = __int_as_float(e0.y);
#pragma unroll
                for (int v = 0; v < V; ++v) acc[v] = fma(w0, (CT)x0[v], acc[v]);
            }
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const float x = hv[v];
                const float ax = fabsf(x);
                const float e = exp_neg(ax);
                const float r = rcp_f(1.0f + e);
                const float pmin = e * r;            // min(P, 1 - P)
                const float pq = pmin * r;           // P (1 - P)
                const float g = (float)((CT)pq * fma((CT)x, (CT)sc.inv_beta_d, (CT)2 * acc[v]));
                gv[v] = g;
                if constexpr (EN) {
                    // own marginal tanh(h/2) = sign(h) (1 - e) r: near h = 0
                    // 1 - e cancels, but its absolute error (about 1e-7)
                    // stays far below the scale of U
                    const float m_own = copysignf((1.0f - e) * r, x);
                    eacc[v] += (float)((CT)m_own * acc[v]);
                    eacc[V + v] += log1p_f(e) + ax * pmin;
                }
                const float nh = adam_update(x, g, m1v[v], m2v[v], sc);
                hv[v] = nh;
                mnew[v] = tanh_half(nh);
            }
            st_state<V, NT>(a.h + sbase, hv);
            st_state<V, NT>(a.m1 + sbase, m1v);
            st_state<V, NT>(a.m2 + sbase, m2v);
            st_marg<MT, V>(mn + base, mnew);
            if (a.grad) st_f32<V>(a.grad + base, gv);
        }
    }
    if constexpr (EN) {
        extern __shared__ double lds_d[];
        double ed[2 * V];
#pragma unroll
        for (int k = 0; k < 2 * V; ++k) ed[k] = (double)eacc[k];
        block_reduce_store<double, 2 * V>(ed, ti, a.lanes_log2, lds_d, [&](int k, int l, double s) {
            const int term = k / V, v = k % V;
            const int r = (seg * ti.L + l) * V + v;
            if (r < R) a.epart[((size_t)tile.slot * 2 + term) * R + r] = s;
        });
    }
}

// ======================================================= bMinCut step =====
// Potts, q states per node, softmax marginals.  With Phi_i(s) = sum_j W_ij
// P_j(s) and C~(s) the centred column sum of the current marginals:
//   A(s) = -2 Phi_i(s) + 2 lam [C~(s) - P_i(s)] + h_i(s) / beta
//   g_i(s) = P_i(s) [A(s) - sum_s' P_i(s') A(s')]
// This equals the chain rule applied to the explicit bMinCut gradient: the
// terms (ln P + 1)/beta and the column-sum centring differ from h/beta and
// C~ by per-(node, replica) constants, which the chain rule removes exactly.
// Energies per replica: [sum_i (sum_j W_ij - P_i.Phi_i), sum_i |P_i|^2,
// -sum_i P_i.ln P_i].  Column sums of the new marginals go out as 2^-40
// fixed point.
// Up to q = 16 each lane keeps its running column sums and energies in its
// own LDS slots (q + 3 doubles per thread, potts_step_lds), and a row's h,
// m1, m2 are loaded after its gather: the registers go to the neighbour rows
// in flight (at q = 8: 121 VGPRs, 4 waves per SIMD, instead of 164 and 3).
// The sums are formed in the same order either way.
template <int Q, typename MT, bool EN, bool NT>
__global__ void __launch_bounds__(step_max_threads(KIND_BMINCUT, Q)) potts_step_kernel(StepArgs a)
{
    const Tile tile = a.tiles[blk_tile(a.seg_major)];
    const int seg = blk_seg(a.seg_major);
    const TeamIdx ti = team_idx(a.lanes_log2);
    const int R = a.R;
    const int r = seg * ti.L + ti.tl;   // replica of this lane
    const bool act = r < R;
    const int RQ = R * Q;
    const MT* __restrict__ mc = static_cast<const MT*>(a.marg_cur);
    MT* __restrict__ mn = static_cast<MT*>(a.marg_nxt);
    const StepScalars sc = a.sc;
    // Phi accumulates in double up to q = 8 (at larger q the registers would
    // not hold it) and the gradient terms combine in double, for either
    // marginal type: the bfloat16 copy changes only the values gathered
    using AccT = typename std::conditional<(Q <= 8), double, float>::type;
    using CT = double;
    constexpr bool LA = potts_lds_acc(Q);
    extern __shared__ double lds_d[];
    const int nthr = blockDim.x, tid = threadIdx.x;
    // LA: slot [s][tid] of cs_l holds column sum s, slot [k][tid] of ea_l energy k
    long long* cs_l = reinterpret_cast<long long*>(lds_d);
    double* ea_l = lds_d + (size_t)Q * nthr;
    AccT ctr[LA ? 1 : Q];
    double eacc[3] = {0.0, 0.0, 0.0};
    long long cs[Q];
#pragma unroll
    for (int s = 0; s < Q; ++s) cs[s] = 0;
    if constexpr (LA) {
#pragma unroll
        for (int s = 0; s < Q; ++s) cs_l[s * nthr + tid] = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) ea_l[k * nthr + tid] = 0.0;
    }
    if (act) {
        const double* ctp = a.ctil + ((size_t)tile.inst * R + r) * Q;
        if constexpr (!LA) {
#pragma unroll
            for (int s = 0; s < Q; ++s) ctr[s] = (AccT)ctp[s];
        }
        for (int i = tile.row_begin + ti.team; i < tile.row_end; i += ti.teams) {
            const size_t base = ((size_t)i * R + r) * Q;
            const size_t sbase = (size_t)i * a.srow + (size_t)r * Q;   // h, m1, m2 rows
            float hv[Q], m1v[Q], m2v[Q];
            if constexpr (!LA) {
                ld_state<Q, NT>(a.h + sbase, hv);
                ld_state<Q, NT>(a.m1 + sbase, m1v);
                ld_state<Q, NT>(a.m2 + sbase, m2v);
            }
            AccT phi[Q];
#pragma unroll
            for (int s = 0; s < Q; ++s) phi[s] = (AccT)0;
            int64_t k = a.row_off[i];
            const int64_t kend = a.row_off[i + 1];
            for (; k + 8 <= kend; k += 8) {
                int2 e[8];
                float x[8][Q];
#pragma unroll
                for (int u = 0; u < 8; ++u) e[u] = a.adj[k + u];
#pragma unroll
                for (int u = 0; u < 8; ++u) ld_marg<MT, Q>(mc + (size_t)e[u].x * RQ + (size_t)r * Q, x[u]);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const AccT w = (AccT)__int_as_float(e[u].y);
#pragma unroll
                    for (int s = 0; s < Q; ++s) phi[s] = fma(w, (AccT)x[u][s], phi[s]);
                }
            }
            for (; k + 4 <= kend; k += 4) {
                const int2 e0 = a.adj[k], e1 = a.adj[k + 1], e2 = a.adj[k + 2], e3 = a.adj[k + 3];
                float x0[Q], x1[Q], x2[Q], x3[Q];
                ld_marg<MT, Q>(mc + (size_t)e0.x * RQ + (size_t)r * Q, x0);
                ld_marg<MT, Q>(mc + (size_t)e1.x * RQ + (size_t)r * Q, x1);
                ld_marg<MT, Q>(mc + (size_t)e2.x * RQ + (size_t)r * Q, x2);
                ld_marg<MT, Q>(mc + (size_t)e3.x * RQ + (size_t)r * Q, x3);
                const AccT w0 = (AccT)__int_as_float(e0.y), w1 = (AccT)__int_as_float(e1.y);
                const AccT w2 = (AccT)__int_as_float(e2.y), w3 = (AccT)__int_as_float(e3.y);
#pragma unroll
                for (int s = 0; s < Q; ++s) {
                    phi[s] = fma(w0, (AccT)x0[s], phi[s]);
                    phi[s] = fma(w1, (AccT)x1[s], phi[s]);
                    phi[s] = fma(w2, (AccT)x2[s], phi[s]);
                    phi[s] = fma(w3, (AccT)x3[s], phi[s]);
                }
            }
            for (; k + 2 <= kend; k += 2) {
                const int2 e0 = a.adj[k], e1 = a.adj[k + 1];
                float x0[Q], x1[Q];
                ld_marg<MT, Q>(mc + (size_t)e0.x * RQ + (size_t)r * Q, x0);
                ld_marg<MT, Q>(mc + (size_t)e1.x * RQ + (size_t)r * Q, x1);
                const AccT w0 = (AccT)__int_as_float(e0.y), w1 = (AccT)__int_as_float(e1.y);
#pragma unroll
                for (int s = 0; s < Q; ++s) {
                    phi[s] = fma(w0, (AccT)x0[s], phi[s]);
                    phi[s] = fma(w1, (AccT)x1[s], phi[s]);
                }
            }
            for (; k < kend; ++k) {
                const int2 e0 = a.adj[k];
                float x0[Q];
                ld_marg<MT, Q>(mc + (size_t)e0.x * RQ + (size_t)r * Q, x0);
                const AccT w0 = (AccT)__int_as_float(e0.y);
#pragma unroll
                for (int s = 0; s < Q; ++s) phi[s] = fma(w0, (AccT)x0[s], phi[s]);
            }
            AccT ct[Q];
            if constexpr (LA) {
                ld_state<Q, NT>(a.h + sbase, hv);
                ld_state<Q, NT>(a.m1 + sbase, m1v);
                ld_state<Q, NT>(a.m2 + sbase, m2v);
#pragma unroll
                for (int s = 0; s < Q; ++s) ct[s] = (AccT)ctp[s];
            } else {
#pragma unroll
                for (int s = 0; s < Q; ++s) ct[s] = ctr[LA ? 0 : s];
            }
            // softmax of the current fields
            float mx = hv[0];
#pragma unroll
            for (int s = 1; s < Q; ++s) mx = fmaxf(mx, hv[s]);
            float P[Q], Z = 0.0f;
#pragma unroll
            for (int s = 0; s < Q; ++s) { P[s] = exp_neg(mx - hv[s]); Z += P[s]; }
            const float invZ = rcp_f(Z);
#pragma unroll
            for (int s = 0; s < Q; ++s) P[s] *= invZ;
            // gradient terms combined in double: A(s) - sum_s' P(s') A(s') is a
            // small difference of large terms once the marginals settle
            // (A is formed twice rather than stored: fewer registers at large q).
            // The mean is normalised by the sum of the float32 marginals, so
            // their rounding perturbs only the weights, by a relative amount,
            // and the error scales with the spread of A, not its size.
            // node weight V_i scales the balance term: 2 lam V_i [C~(s) - V_i P_i(s)]
            const float vw = a.nw ? (float)a.nw[i] : 1.0f;
            const CT lam2 = (CT)2 * (CT)sc.lam_d * (CT)vw, ib = (CT)sc.inv_beta_d;
            auto Aof = [&](int s) {
                return (CT)-2 * (CT)phi[s] + lam2 * ((CT)ct[s] - (CT)vw * (CT)P[s]) + ((CT)hv[s] - (CT)mx) * ib;
            };
            CT avg = 0, psum = 0;
#pragma unroll
            for (int s = 0; s < Q; ++s) {
                avg = fma((CT)P[s], Aof(s), avg);
                psum += (CT)P[s];
            }
            avg /= psum;
            float gv[Q];
#pragma unroll
            for (int s = 0; s < Q; ++s) gv[s] = (float)((Aof(s) - avg) * (CT)P[s]);
            if constexpr (EN) {
                const float lz = __builtin_amdgcn_logf(Z) * 0.693147180559945309f;   // ln Z, Z in [1, q]
                double dot = 0.0;
                float sq = 0.0f, ent = 0.0f;
#pragma unroll
                for (int s = 0; s < Q; ++s) {
                    dot = fma((double)P[s], (double)phi[s], dot);
                    sq = fmaf(vw * P[s], vw * P[s], sq);
                    ent = fmaf(-P[s], hv[s] - mx - lz, ent);
                }
                const double e3[3] = {(double)a.wdeg[i] - dot, (double)sq, (double)ent};
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    if constexpr (LA) ea_l[k * nthr + tid] += e3[k];
                    else eacc[k] += e3[k];
                }
            }
            // Adam, then the softmax of the new fields
#pragma unroll
            for (int s = 0; s < Q; ++s) hv[s] = adam_update(hv[s], gv[s], m1v[s], m2v[s], sc);
            // the new softmax in double: the stored marginals and their
            // column-sum contributions (the rounding of float32 marginals,
            // summed over all nodes, would carry into the balance term)
            if constexpr (LA) {
#pragma unroll
                for (int s = 0; s < Q; ++s) cs[s] = 0;
            }
            float Pn[Q];
            softmax_colsum<Q>(hv, cs, (double)vw, Pn);
            if constexpr (LA) {
#pragma unroll
                for (int s = 0; s < Q; ++s) cs_l[s * nthr + tid] += cs[s];
            }
            st_state<Q, NT>(a.h + sbase, hv);
            st_state<Q, NT>(a.m1 + sbase, m1v);
            st_state<Q, NT>(a.m2 + sbase, m2v);
            st_marg<MT, Q>(mn + base, Pn);
            if (a.grad) st_f32<Q>(a.grad + base, gv);
        }
    }
    if constexpr (LA) {
        // every lane reads its own slots before the reduction reuses the LDS
#pragma unroll
        for (int s = 0; s < Q; ++s) cs[s] = cs_l[s * nthr + tid];
#pragma unroll
        for (int k = 0; k < 3; ++k) eacc[k] = ea_l[k * nthr + tid];
        __syncthreads();
    }
    block_reduce_store<long long, Q>(cs, ti, a.lanes_log2, reinterpret_cast<long long*>(lds_d),
                                     [&](int s, int l, long long v) {
                                         const int rr = seg * ti.L + l;
                                         if (rr < R) a.cpart[((size_t)tile.slot * R + rr) * Q + s] = v;
                                     });
    if constexpr (EN) {
        block_reduce_store<double, 3>(eacc, ti, a.lanes_log2, lds_d, [&](int k, int l, double s) {
            const int rr = seg * ti.L + l;
            if (rr < R) a.epart[((size_t)tile.slot * 3 + k) * R + rr] = s;
        });
    }
}

// ======================================================= Max-k-SAT step ===
// Variable-centric: every incidence (m, i) of variable i stores the clause's
// other literals.  With u = probability that a literal is false and
// c_mi = prod_{k in m, k != i} u_mk (the cavity product, formed from the
// others, never by division):
//   d_i = sum_{m ∋ i} (literal positive ? -1 : +1) c_mi
//   g_i = P_i (1 - P_i) [d_i + h_i / beta]
// Energies per replica: [sum over owner incidences of prod_{k in m} u_mk,
// sum_i H2(P_i)]; each clause has exactly one owner incidence.
template <int W>
struct SatRec;
template <>
struct SatRec<2> {
    using T = int2;
};
template <>
struct SatRec<3> {
    using T = int4;
};

template <int V, typename MT, int W, bool EN, bool NT>
__global__ void __launch_bounds__(step_max_threads(KIND_MAXSAT, V)) sat_step_kernel(StepArgs a)
{
    const Tile tile = a.tiles[blk_tile(a.seg_major)];
    const int seg = blk_seg(a.seg_major);
    const TeamIdx ti = team_idx(a.lanes_log2);
    const int R = a.R;
    const int rb = (seg * ti.L + ti.tl) * V;
    const bool act = rb < R;
    const MT* __restrict__ mc = static_cast<const MT*>(a.marg_cur);
    MT* __restrict__ mn = static_cast<MT*>(a.marg_nxt);
    const StepScalars sc = a.sc;
    // the clause sums and the gradient combination are formed in double for
    // either marginal type
    using CT = double;
    float eacc[2 * V];
#pragma unroll
    for (int k = 0; k < 2 * V; ++k) eacc[k] = 0.0f;
    using Rec = typename SatRec<W>::T;
    const Rec* __restrict__ inc = reinterpret_cast<const Rec*>(W == 2 ? (const void*)a.inc2 : (const void*)a.inc4);

    if (act) {
        for (int i = tile.row_begin + ti.team; i < tile.row_end; i += ti.teams) {
            const size_t base = (size_t)i * R + rb;
            const size_t sbase = (size_t)i * a.srow + rb;   // h, m1, m2 rows
            float hv[V], m1v[V], m2v[V];
            ld_state<V, NT>(a.h + sbase, hv);
            ld_state<V, NT>(a.m1 + sbase, m1v);
            ld_state<V, NT>(a.m2 + sbase, m2v);
            // the variable's own min(P, 1 - P) and side, for the clause
            // energies at owner incidences
            float own_small[V];
            bool own_hi[V];
            if constexpr (EN) {
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const float e = exp_neg(fabsf(hv[v]));
                    own_small[v] = e * rcp_f(1.0f + e);
                    own_hi[v] = hv[v] > 0.0f;
                }
            }
            CT d[V];
#pragma unroll
            for (int v = 0; v < V; ++v) d[v] = (CT)0;
            // literals of an incidence record: the other variables with their
            // signs, the own sign, and whether this is the clause's owner
            auto decode = [&](const Rec& rec, uint32_t (&lit)[W], bool& own_pos, bool& owner) {
                if constexpr (W == 2) {
                    lit[0] = (uint32_t)rec.x; lit[1] = (uint32_t)rec.y;
                    own_pos = (lit[0] & SAT_FLAG) != 0;
                    owner = (lit[1] & SAT_FLAG) != 0;
                } else {
                    lit[0] = (uint32_t)rec.x; lit[1] = (uint32_t)rec.y; lit[2] = (uint32_t)rec.z;
                    own_pos = (rec.w & 1) != 0;
                    owner = (rec.w & 2) != 0;
                }
            };
            // the cavity product of one incidence from its gathered rows, added
            // to d (and to the energy at the owner) in incidence order; no
            // branches, so that a round's loads all issue before its waits
            auto combine = [&](const uint32_t (&lit)[W], bool own_pos, bool owner, const float (&x)[W][V]) {
                float c[V];
#pragma unroll
                for (int v = 0; v < V; ++v) c[v] = sat_u_bits(x[0][v], lit[0] & SAT_POS);
#pragma unroll
                for (int s = 1; s < W; ++s)
#pragma unroll
                    for (int v = 0; v < V; ++v) c[v] *= sat_u_bits(x[s][v], lit[s] & SAT_POS);
                const float sg = own_pos ? -1.0f : 1.0f;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    d[v] += (CT)(sg * c[v]);
                    if constexpr (EN) {
                        const float uo = (own_pos == own_hi[v]) ? own_small[v] : 1.0f - own_small[v];
                        eacc[v] += owner ? uo * c[v] : 0.0f;
                    }
                }
            };
            // an unused slot (SAT_NONE, a negative literal) reads row n, which
            // holds -0.0: a literal that is false with probability 1
            auto gather = [&](const uint32_t (&lit)[W], float (&x)[W][V]) {
#pragma unroll
                for (int s = 0; s < W; ++s) {
                    const uint32_t var = min(lit[s] & SAT_VAR_MASK, (uint32_t)a.n);
                    ld_marg<MT, V>(mc + (size_t)var * R + rb, x[s]);
                }
            };
            int64_t k = a.row_off[i];
            const int64_t kend = a.row_off[i + 1];
            // NI incidences per round: their records, then all their rows, are
            // in flight together
            constexpr int NI = V <= 2 ? 4 : 2;
            for (; k + NI <= kend; k += NI) {
                Rec rr[NI];
                uint32_t l[NI][W];
                bool po[NI], ow[NI];
                float x[NI][W][V];
#pragma unroll
                for (int u = 0; u < NI; ++u) rr[u] = inc[k + u];
#pragma unroll
                for (int u = 0; u < NI; ++u) decode(rr[u], l[u], po[u], ow[u]);
#pragma unroll
                for (int u = 0; u < NI; ++u) gather(l[u], x[u]);
#pragma unroll
                for (int u = 0; u < NI; ++u) combine(l[u], po[u], ow[u], x[u]);
            }
            for (; k < kend; ++k) {
                uint32_t l0[W];
                bool p0, o0;
                decode(inc[k], l0, p0, o0);
                float x0[W][V];
                gather(l0, x0);
                combine(l0, p0, o0, x0);
            }
            float gv[V], snew[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const float x = hv[v];
                const float ax = fabsf(x);
                const float e = exp_neg(ax);
                const float r = rcp_f(1.0f + e);
                const float pmin = e * r;            // min(P, 1 - P)
                const float pq = pmin * r;           // P (1 - P)
                const float g = (float)((CT)sc.gamma_d * ((CT)pq * fma((CT)x, (CT)sc.inv_beta_d, d[v])));
                gv[v] = g;
                if constexpr (EN) eacc[V + v] += log1p_f(e) + ax * pmin;
                const float nh = adam_update(x, g, m1v[v], m2v[v], sc);
                hv[v] = nh;
                snew[v] = sat_encode(nh);
            }
            st_state<V, NT>(a.h + sbase, hv);
            st_state<V, NT>(a.m1 + sbase, m1v);
            st_state<V, NT>(a.m2 + sbase, m2v);
            st_marg<MT, V>(mn + base, snew);
            if (a.grad) st_f32<V>(a.grad + base, gv);
        }
    }
    if constexpr (EN) {
        extern __shared__ double lds_d[];
        double ed[2 * V];
#pragma unroll
        for (int k = 0; k < 2 * V; ++k) ed[k] = (double)eacc[k];
        block_reduce_store<double, 2 * V>(ed, ti, a.lanes_log2, lds_d, [&](int k, int l, double s) {
            const int term = k / V, v = k % V;
            const int r = (seg * ti.L + l) * V + v;
            if (r < R) a.epart[((size_t)tile.slot * 2 + term) * R + r] = s;
        });
    }
}

// ================================================== marginal initialisation
// Writes the marginal copy of the current fields (m = tanh(h/2), the SAT
// encoding, or the softmax) into marg_nxt; for Potts also the column-sum
// partials of those marginals.
template <typename MT>
__global__ void init_q1_kernel(int kind, const float* __restrict__ h, int32_t R, int64_t srow, MT* __restrict__ out,
                               size_t count)
{
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (size_t)gridDim.x * blockDim.x) {
        const float hv = h[(k / R) * srow + k % R];
        float x[1] = {kind == KIND_MAXSAT ? sat_encode(hv) : tanh_half(hv)};
        st_marg<MT, 1>(out + k, x);
    }
}

template <int Q, typename MT>
__global__ void __launch_bounds__(step_max_threads(KIND_BMINCUT, Q)) potts_init_kernel(StepArgs a)
{
    const Tile tile = a.tiles[blk_tile(a.seg_major)];
    const int seg = blk_seg(a.seg_major);
    const TeamIdx ti = team_idx(a.lanes_log2);
    const int R = a.R;
    const int r = seg * ti.L + ti.tl;
    const bool act = r < R;
    MT* __restrict__ mn = static_cast<MT*>(a.marg_nxt);
    long long cs[Q];
#pragma unroll
    for (int s = 0; s < Q; ++s) cs[s] = 0;
    if (act) {
        for (int i = tile.row_begin + ti.team; i < tile.row_end; i += ti.teams) {
            const size_t base = ((size_t)i * R + r) * Q;
            const size_t sbase = (size_t)i * a.srow + (size_t)r * Q;   // h, m1, m2 rows
            float hv[Q];
            ld_f32<Q>(a.h + sbase, hv);
            float P[Q];
            softmax_colsum<Q>(hv, cs, a.nw ? (double)a.nw[i] : 1.0, P);
            st_marg<MT, Q>(mn + base, P);
        }
    }
    extern __shared__ double lds_d[];
    block_reduce_store<long long, Q>(cs, ti, a.lanes_log2, reinterpret_cast<long long*>(lds_d),
                                     [&](int s, int l, long long v) {
                                         const int rr = seg * ti.L + l;
                                         if (rr < R) a.cpart[((size_t)tile.slot * R + rr) * Q + s] = v;
                                     });
}

// ============================================== segmented tile reductions ==
// out[seg][c] = sum_{t in [seg_off[seg], seg_off[seg+1])} part[t][c], in a
// fixed order: eight sub-sums over t = t0+sub, t0+sub+8, ..., then sub 0..7.
template <typename T>
__global__ void __launch_bounds__(256) seg_reduce_kernel(const T* __restrict__ part, int cols,
                                                         const int32_t* __restrict__ seg_off,
                                                         T* __restrict__ out)
{
    __shared__ T lds[256];
    const int seg = blockIdx.x;
    const int c = blockIdx.y * 32 + (threadIdx.x & 31);
    const int sub = threadIdx.x >> 5;
    const int t0 = seg_off[seg], t1 = seg_off[seg + 1];
    T acc = 0;
    if (c < cols)
        for (int t = t0 + sub; t < t1; t += 8) acc += part[(size_t)t * cols + c];
    lds[threadIdx.x] = acc;
    __syncthreads();
    if (sub == 0 && c < cols) {
        T v = lds[threadIdx.x];
#pragma unroll
        for (int s = 1; s < 8; ++s) v += lds[s * 32 + threadIdx.x];
        out[(size_t)seg * cols + c] = v;
    }
}

template <typename T>
static hipError_t seg_reduce2(const T* part, int cols, const int32_t* chunk_off, int n_chunks,
                              const int32_t* inst_chunk_off, int n_inst, T* tmp, T* out, hipStream_t st)
{
    (void)hipGetLastError();
    dim3 g1(n_chunks, (cols + 31) / 32);
    seg_reduce_kernel<T><<<g1, 256, 0, st>>>(part, cols, chunk_off, tmp);
    dim3 g2(n_inst, (cols + 31) / 32);
    seg_reduce_kernel<T><<<g2, 256, 0, st>>>(tmp, cols, inst_chunk_off, out);
    return hipGetLastError();
}

// Energies straight from the per-tile partials [tile][NE][R], one launch:
// block (inst, replica group of 32) sums the instance's tiles in 8 strided
// sub-sums added in fixed order, then forms U, S, F.  For instances of few
// tiles, where the two-stage reduction and the combination cost three
// launches for a few thousand values.
template <int NE>
__global__ void __launch_bounds__(256) energy_finish_kernel(int kind, int R, int q, const double* __restrict__ part,
                                                            const int32_t* __restrict__ chunk_off,
                                                            const int32_t* __restrict__ inst_chunk_off,
                                                            const double* __restrict__ wtot,
                                                            const double* __restrict__ csum, double lam,
                                                            double beta, double* __restrict__ eout)
{
    __shared__ double lds[NE][256];
    const int inst = blockIdx.x;
    const int r = blockIdx.y * 32 + (threadIdx.x & 31);
    const int sub = threadIdx.x >> 5;
    const int t0 = chunk_off[inst_chunk_off[inst]], t1 = chunk_off[inst_chunk_off[inst + 1]];
    double acc[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) acc[k] = 0.0;
    if (r < R)
        for (int t = t0 + sub; t < t1; t += 8)
#pragma unroll
            for (int k = 0; k < NE; ++k) acc[k] += part[((size_t)t * NE + k) * R + r];
#pragma unroll
    for (int k = 0; k < NE; ++k) lds[k][threadIdx.x] = acc[k];
    __syncthreads();
    if (sub == 0 && r < R) {
        double x[NE];
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            double v = lds[k][threadIdx.x];
            for (int s = 1; s < 8; ++s) v += lds[k][s * 32 + threadIdx.x];
            x[k] = v;
        }
        // U, S, F as energy_combine_kernel forms them
        double U, S;
        if (kind == KIND_MAXCUT) {
            U = -wtot[inst] + 0.5 * x[0];
            S = x[1];
        } else if (kind == KIND_MAXSAT) {
            U = x[0];
            S = x[1];
        } else {
            const double* C = csum + ((size_t)inst * R + r) * q;
            double c2 = 0.0;
            for (int s = 0; s < q; ++s) c2 += C[s] * C[s];
            U = x[0] + lam * (c2 - x[1]);
            S = x[NE - 1];
        }
        double* o = eout + (size_t)inst * 3 * R;
        o[r] = U;
        o[R + r] = S;
        o[2 * R + r] = U - S / beta;
    }
}

// energies: raw[inst][NE][R] -> eout[inst][3][R] = U, S, F
__global__ void energy_combine_kernel(int kind, int R, int q, int n_inst, const double* __restrict__ raw,
                                      const double* __restrict__ wtot, const double* __restrict__ csum,
                                      double lam, double beta, double* __restrict__ eout)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_inst * R) return;
    const int inst = idx / R, r = idx % R;
    double U, S;
    if (kind == KIND_MAXCUT) {
        const double* x = raw + (size_t)inst * 2 * R;
        U = -wtot[inst] + 0.5 * x[r];
        S = x[R + r];
    } else if (kind == KIND_MAXSAT) {
        const double* x = raw + (size_t)inst * 2 * R;
        U = x[r];
        S = x[R + r];
    } else {
        const double* x = raw + (size_t)inst * 3 * R;
        const double* C = csum + ((size_t)inst * R + r) * q;
        double c2 = 0.0;
        for (int s = 0; s < q; ++s) c2 += C[s] * C[s];
        U = x[r] + lam * (c2 - x[R + r]);
        S = x[2 * R + r];
    }
    double* o = eout + (size_t)inst * 3 * R;
    o[r] = U;
    o[R + r] = S;
    o[2 * R + r] = U - S / beta;
}

// column sums: fixed point -> C (double) and centred C~ (float)
__global__ void colsum_combine_kernel(int R, int q, int n_inst, const long long* __restrict__ fx, double scale,
                                      double* __restrict__ csum, double* __restrict__ ctil)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_inst * R) return;
    const long long* x = fx + (size_t)idx * q;
    double mean = 0.0;
    for (int s = 0; s < q; ++s) {
        const double c = (double)x[s] * scale;
        csum[(size_t)idx * q + s] = c;
        mean += c;
    }
    mean /= q;
    for (int s = 0; s < q; ++s) ctil[(size_t)idx * q + s] = csum[(size_t)idx * q + s] - mean;
}

// ================================================ read-out & evaluation ===
// sigma[i][r] = argmax_s h_i^r(s), ties to the lowest state; one logit: h > 0.
__global__ void round_kernel(int kind, int32_t n, int32_t R, int32_t q, const float* __restrict__ h, int64_t srow,
                             uint8_t* __restrict__ sigma)
{
    const size_t count = (size_t)n * R;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (size_t)gridDim.x * blockDim.x) {
        const size_t i = k / R, r = k % R;
        if (kind != KIND_BMINCUT) {
            sigma[k] = h[i * srow + r] > 0.0f ? 1 : 0;
        } else {
            const float* x = h + i * srow + r * q;
            int best = 0;
            float bv = x[0];
            for (int s = 1; s < q; ++s)
                if (x[s] > bv) { bv = x[s]; best = s; }
            sigma[k] = (uint8_t)best;
        }
    }
}

// Rows of w floats between arrays with row strides ds and ss (floats), and
// zeros into z1 and z2 (row stride ds) where they are given; src null copies
// nothing.  Four floats per lane when every stride, w and pointer allow it.
template <typename V>
__global__ void rows_kernel(int32_t n, int64_t w, float* __restrict__ dst, int64_t ds, const float* __restrict__ src,
                            int64_t ss, float* __restrict__ z1, float* __restrict__ z2)
{
    constexpr int L = sizeof(V) / sizeof(float);
    const int64_t wv = w / L;
    const size_t count = (size_t)n * wv;
    const V zero{};
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (size_t)gridDim.x * blockDim.x) {
        const size_t i = k / wv, c = (k % wv) * L;
        const size_t od = i * ds + c;
        if (src) *reinterpret_cast<V*>(dst + od) = *reinterpret_cast<const V*>(src + i * ss + c);
        if (z1) *reinterpret_cast<V*>(z1 + od) = zero;
        if (z2) *reinterpret_cast<V*>(z2 + od) = zero;
    }
}

// host [R][n] int32 -> device [n][R] uint8
__global__ void transpose_sigma_kernel(int32_t n, int32_t R, const int32_t* __restrict__ in, uint8_t* __restrict__ out)
{
    const size_t count = (size_t)n * R;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (size_t)gridDim.x * blockDim.x) {
        const size_t i = k / R, r = k % R;
        out[k] = (uint8_t)in[r * (size_t)n + i];
    }
}

// Ordered cut sum_{j in N(i)} W_ij [sigma_i != sigma_j] per replica (graphs),
// group sizes (bMinCut: sums of the node weights nw, 1 each when null), or
// unsatisfied clauses counted at owner incidences (Max-k-SAT).  One lane per
// replica.
template <int Q>
__global__ void __launch_bounds__(1024) eval_graph_kernel(const int64_t* __restrict__ row_off, const int2* __restrict__ adj,
                                                         const int32_t* __restrict__ nw, const Tile* __restrict__ tiles,
                                                         int32_t R, int lanes_log2, const uint8_t* __restrict__ sigma,
                                                         double* __restrict__ vpart, int* __restrict__ spart)
{
    const Tile tile = tiles[blockIdx.x];
    const TeamIdx ti = team_idx(lanes_log2);
    const int r = blockIdx.y * ti.L + ti.tl;
    const bool act = r < R;
    double acc[1] = {0.0};
    int cnt[Q];
#pragma unroll
    for (int s = 0; s < Q; ++s) cnt[s] = 0;
    if (act) {
        for (int i = tile.row_begin + ti.team; i < tile.row_end; i += ti.teams) {
            const uint8_t si = sigma[(size_t)i * R + r];
            if constexpr (Q > 1) {
                const int vi = nw ? nw[i] : 1;
#pragma unroll
                for (int s = 0; s < Q; ++s) cnt[s] += (si == s) ? vi : 0;
            }
            int64_t k = row_off[i];
            const int64_t kend = row_off[i + 1];
            // rounds of up to eight neighbours in flight, summed in CSR order
            for (; k < kend; k += 8) {
                const int nb = (int)min((int64_t)8, kend - k);
                int2 e[8];
                uint8_t sj[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (u < nb) e[u] = adj[k + u];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (u < nb) sj[u] = sigma[(size_t)e[u].x * R + r];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (u < nb && sj[u] != si) acc[0] += (double)__int_as_float(e[u].y);
            }
        }
    }
    extern __shared__ double lds_d[];
    block_reduce_store<double, 1>(acc, ti, lanes_log2, lds_d, [&](int, int l, double s) {
        const int rr = blockIdx.y * ti.L + l;
        if (rr < R) vpart[(size_t)tile.slot * R + rr] = s;
    });
    if constexpr (Q > 1) {
        block_reduce_store<int, Q>(cnt, ti, lanes_log2, reinterpret_cast<int*>(lds_d), [&](int s, int l, int v) {
            const int rr = blockIdx.y * ti.L + l;
            if (rr < R) spart[((size_t)tile.slot * R + rr) * Q + s] = v;
        });
    }
}

// MaxCut with R a multiple of 4: the ordered cut sums of eval_graph_kernel<1>
// for four replicas per lane, with one 32-bit load of their four sigma bytes
// per neighbour.
__global__ void __launch_bounds__(1024) eval_cut4_kernel(const int64_t* __restrict__ row_off,
                                                        const int2* __restrict__ adj, const Tile* __restrict__ tiles,
                                                        int32_t R, int lanes_log2, const uint8_t* __restrict__ sigma,
                                                        double* __restrict__ vpart)
{
    const Tile tile = tiles[blockIdx.x];
    const TeamIdx ti = team_idx(lanes_log2);
    const int r0 = 4 * (blockIdx.y * ti.L + ti.tl);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (r0 < R) {
        for (int i = tile.row_begin + ti.team; i < tile.row_end; i += ti.teams) {
            const uint32_t si = *reinterpret_cast<const uint32_t*>(sigma + (size_t)i * R + r0);
            int64_t k = row_off[i];
            const int64_t kend = row_off[i + 1];
            // rounds of up to eight neighbours in flight, summed in CSR order
            for (; k < kend; k += 8) {
                const int nb = (int)min((int64_t)8, kend - k);
                int2 e[8];
                uint32_t sj[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (u < nb) e[u] = adj[k + u];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (u < nb) sj[u] = *reinterpret_cast<const uint32_t*>(sigma + (size_t)e[u].x * R + r0);
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (u < nb) {
                        const uint32_t d = si ^ sj[u];
                        const double w = (double)__int_as_float(e[u].y);
#pragma unroll
                        for (int b = 0; b < 4; ++b)
                            if ((d >> (8 * b)) & 0xffu) acc[b] += w;
                    }
            }
        }
    }
    extern __shared__ double lds_d[];
    block_reduce_store<double, 4>(acc, ti, lanes_log2, lds_d, [&](int b, int l, double v) {
        const int rr = 4 * (blockIdx.y * ti.L + l) + b;
        if (rr < R) vpart[(size_t)tile.slot * R + rr] = v;
    });
}

template <int W>
__global__ void __launch_bounds__(1024) eval_sat_kernel(const int64_t* __restrict__ row_off, const void* __restrict__ incv,
                                                       const Tile* __restrict__ tiles, int32_t R, int lanes_log2,
                                                       const uint8_t* __restrict__ sigma, double* __restrict__ vpart)
{
    using Rec = typename SatRec<W>::T;
    const Rec* inc = reinterpret_cast<const Rec*>(incv);
    const Tile tile = tiles[blockIdx.x];
    const TeamIdx ti = team_idx(lanes_log2);
    const int r = blockIdx.y * ti.L + ti.tl;
    const bool act = r < R;
    double acc[1] = {0.0};
    if (act) {
        for (int i = tile.row_begin + ti.team; i < tile.row_end; i += ti.teams) {
            const uint8_t si = sigma[(size_t)i * R + r];
            for (int64_t k = row_off[i]; k < row_off[i + 1]; ++k) {
                const Rec rec = inc[k];
                uint32_t lit[W];
                bool own_pos, owner;
                if constexpr (W == 2) {
                    lit[0] = (uint32_t)rec.x; lit[1] = (uint32_t)rec.y;
                    own_pos = (lit[0] & SAT_FLAG) != 0;
                    owner = (lit[1] & SAT_FLAG) != 0;
                } else {
                    lit[0] = (uint32_t)rec.x; lit[1] = (uint32_t)rec.y; lit[2] = (uint32_t)rec.z;
                    own_pos = (rec.w & 1) != 0;
                    owner = (rec.w & 2) != 0;
                }
                if (!owner) continue;
                bool all_false = own_pos ? (si == 0) : (si == 1);
#pragma unroll
                for (int s = 0; s < W; ++s) {
                    const uint32_t var = lit[s] & SAT_VAR_MASK;
                    if (var != SAT_NONE) {
                        const uint8_t sv = sigma[(size_t)var * R + r];
                        const bool pos = (lit[s] & SAT_POS) != 0;
                        all_false = all_false && (pos ? (sv == 0) : (sv == 1));
                    }
                }
                acc[0] += all_false ? 1.0 : 0.0;
            }
        }
    }
    extern __shared__ double lds_d[];
    block_reduce_store<double, 1>(acc, ti, lanes_log2, lds_d, [&](int, int l, double s) {
        const int rr = blockIdx.y * ti.L + l;
        if (rr < R) vpart[(size_t)tile.slot * R + rr] = s;
    });
}

// values[inst][R] (double) and sizes[inst][R][q] (int64 from int) finished
__global__ void sizes_widen_kernel(size_t count, const int* __restrict__ in, long long* __restrict__ out)
{
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (size_t)gridDim.x * blockDim.x)
        out[k] = in[k];
}

// anytime best: best[inst][r] <- better of best and the value just evaluated.
// MaxCut: cut = ordered / 2, larger is better; Max-k-SAT: fewer unsat;
// bMinCut: integer energy 2 cut + lam (sum_s W_s^2 - sum_i V_i^2), lower, with
// W_s the summed node weight of group s (|Pi_s| (|Pi_s| - 1) summed over s for
// unit weights).
__global__ void best_update_kernel(int kind, int R, int n_inst, int q, double lam, const double* __restrict__ v,
                                   const long long* __restrict__ sz, const double* __restrict__ v2,
                                   double* __restrict__ best)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_inst * R) return;
    double score;
    if (kind == KIND_MAXCUT) {
        score = -0.5 * v[idx];
    } else if (kind == KIND_MAXSAT) {
        score = v[idx];
    } else {
        double pen = -v2[idx / R];
        for (int s = 0; s < q; ++s) {
            const double c = (double)sz[(size_t)idx * q + s];
            pen += c * c;   // exact: group weights are below 2^22
        }
        score = v[idx] + lam * pen;   // ordered cut = 2 cut
    }
    if (score < best[idx]) best[idx] = score;
}

// ============================================================ launchers ===
// LDS for block_reduce_store: waves * L * K values of 8 bytes.

template <int V, typename MT, bool NT>
static void launch_maxcut(bool en, dim3 g, dim3 b, int L, const StepArgs& a, hipStream_t st)
{
    const size_t lds = en ? lds_bytes(b.x / 64, L, 2 * V) : 0;
    if (a.adj_pm1) {
        if (en) maxcut_step_kernel<V, MT, true, NT, true><<<g, b, lds, st>>>(a);
        else maxcut_step_kernel<V, MT, false, NT, true><<<g, b, lds, st>>>(a);
    } else {
        if (en) maxcut_step_kernel<V, MT, true, NT, false><<<g, b, lds, st>>>(a);
        else maxcut_step_kernel<V, MT, false, NT, false><<<g, b, lds, st>>>(a);
    }
}
template <int V, typename MT, int W, bool NT>
static void launch_sat(bool en, dim3 g, dim3 b, int L, const StepArgs& a, hipStream_t st)
{
    if (en) sat_step_kernel<V, MT, W, true, NT><<<g, b, lds_bytes(b.x / 64, L, 2 * V), st>>>(a);
    else sat_step_kernel<V, MT, W, false, NT><<<g, b, 0, st>>>(a);
}
template <int Q, typename MT, bool NT>
static void launch_potts(bool en, dim3 g, dim3 b, int L, const StepArgs& a, hipStream_t st)
{
    const size_t lds = potts_step_lds(b.x, L, Q);
    if (en) potts_step_kernel<Q, MT, true, NT><<<g, b, lds, st>>>(a);
    else potts_step_kernel<Q, MT, false, NT><<<g, b, lds, st>>>(a);
}

template <typename MT, bool NT>
static hipError_t launch_step_t(int kind, int vec, const LaunchGeom& geo, int waves, const StepArgs& a,
                                hipStream_t st)
{
    const dim3 g = geo.seg_major ? dim3(geo.nseg, geo.n_tiles) : dim3(geo.n_tiles, geo.nseg);
    const dim3 b(64 * waves);
    const int L = geo.lanes;
    const bool en = a.epart != nullptr;
    if (kind == KIND_MAXCUT) {
        switch (vec) {
        case 1: launch_maxcut<1, MT, NT>(en, g, b, L, a, st); break;
        case 2: launch_maxcut<2, MT, NT>(en, g, b, L, a, st); break;
        case 4: launch_maxcut<4, MT, NT>(en, g, b, L, a, st); break;
        case 8: launch_maxcut<8, MT, NT>(en, g, b, L, a, st); break;
        default: return hipErrorInvalidValue;
        }
    } else if (kind == KIND_MAXSAT) {
        const bool w2 = a.inc2 != nullptr;
        switch (vec) {
        case 1: w2 ? launch_sat<1, MT, 2, NT>(en, g, b, L, a, st) : launch_sat<1, MT, 3, NT>(en, g, b, L, a, st); break;
        case 2: w2 ? launch_sat<2, MT, 2, NT>(en, g, b, L, a, st) : launch_sat<2, MT, 3, NT>(en, g, b, L, a, st); break;
        case 4: w2 ? launch_sat<4, MT, 2, NT>(en, g, b, L, a, st) : launch_sat<4, MT, 3, NT>(en, g, b, L, a, st); break;
        case 8: w2 ? launch_sat<8, MT, 2, NT>(en, g, b, L, a, st) : launch_sat<8, MT, 3, NT>(en, g, b, L, a, st); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (a.q) {
        case 2: launch_potts<2, MT, NT>(en, g, b, L, a, st); break;
        case 4: launch_potts<4, MT, NT>(en, g, b, L, a, st); break;
        case 8: launch_potts<8, MT, NT>(en, g, b, L, a, st); break;
        case 16: launch_potts<16, MT, NT>(en, g, b, L, a, st); break;
        case 32: launch_potts<32, MT, NT>(en, g, b, L, a, st); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_step(int kind, int dtype, int vec, bool nt, const LaunchGeom& g, int waves, const StepArgs& a,
                       hipStream_t st)
{
    (void)hipGetLastError();   // drop stale errors of earlier calls
    if (dtype == 1)
        return nt ? launch_step_t<uint16_t, true>(kind, vec, g, waves, a, st)
                  : launch_step_t<uint16_t, false>(kind, vec, g, waves, a, st);
    return nt ? launch_step_t<float, true>(kind, vec, g, waves, a, st)
              : launch_step_t<float, false>(kind, vec, g, waves, a, st);
}

template <typename MT>
static hipError_t launch_potts_init_t(const LaunchGeom& geo, int waves, const StepArgs& a, hipStream_t st)
{
    const dim3 g = geo.seg_major ? dim3(geo.nseg, geo.n_tiles) : dim3(geo.n_tiles, geo.nseg);
    const dim3 b(64 * waves);
    const size_t lds = lds_bytes(waves, geo.lanes, a.q);
    switch (a.q) {
    case 2: potts_init_kernel<2, MT><<<g, b, lds, st>>>(a); break;
    case 4: potts_init_kernel<4, MT><<<g, b, lds, st>>>(a); break;
    case 8: potts_init_kernel<8, MT><<<g, b, lds, st>>>(a); break;
    case 16: potts_init_kernel<16, MT><<<g, b, lds, st>>>(a); break;
    case 32: potts_init_kernel<32, MT><<<g, b, lds, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static inline int grid_for(size_t count)
{
    const size_t b = (count + 255) / 256;
    return (int)(b < 65536 ? (b ? b : 1) : 65536);
}

hipError_t launch_init_marginals(int kind, int dtype, const LaunchGeom& g, int waves, const StepArgs& a,
                                 size_t count, hipStream_t st)
{
    (void)hipGetLastError();   // drop stale errors of earlier calls
    if (kind == KIND_BMINCUT) {
        if (dtype == 1) return launch_potts_init_t<uint16_t>(g, waves, a, st);
        return launch_potts_init_t<float>(g, waves, a, st);
    }
    if (count == 0) return hipSuccess;
    if (dtype == 1)
        init_q1_kernel<uint16_t><<<grid_for(count), 256, 0, st>>>(kind, a.h, a.R, a.srow,
                                                                 static_cast<uint16_t*>(a.marg_nxt), count);
    else
        init_q1_kernel<float><<<grid_for(count), 256, 0, st>>>(kind, a.h, a.R, a.srow, static_cast<float*>(a.marg_nxt),
                                                              count);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_seg_reduce(const T* part, int cols, const int32_t* chunk_off, int n_chunks,
                             const int32_t* inst_chunk_off, int n_inst, T* tmp, T* out, hipStream_t st)
{
    return seg_reduce2<T>(part, cols, chunk_off, n_chunks, inst_chunk_off, n_inst, tmp, out, st);
}
template hipError_t launch_seg_reduce<double>(const double*, int, const int32_t*, int, const int32_t*, int,
                                              double*, double*, hipStream_t);
template hipError_t launch_seg_reduce<long long>(const long long*, int, const int32_t*, int, const int32_t*, int,
                                                 long long*, long long*, hipStream_t);
template hipError_t launch_seg_reduce<int>(const int*, int, const int32_t*, int, const int32_t*, int, int*, int*,
                                           hipStream_t);

hipError_t launch_energy_finish(int kind, int R, int q, int NE, int n_inst, const double* part,
                                const int32_t* chunk_off, const int32_t* inst_chunk_off, const double* wtot,
                                const double* csum, double lam, double beta, double* eout, hipStream_t st)
{
    (void)hipGetLastError();   // drop stale errors of earlier calls
    const dim3 g(n_inst, (R + 31) / 32);
    if (NE == 2)
        energy_finish_kernel<2><<<g, 256, 0, st>>>(kind, R, q, part, chunk_off, inst_chunk_off, wtot, csum, lam, beta,
                                                   eout);
    else if (NE == 3)
        energy_finish_kernel<3><<<g, 256, 0, st>>>(kind, R, q, part, chunk_off, inst_chunk_off, wtot, csum, lam, beta,
                                                   eout);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_energy_combine(int kind, int R, int q, int n_inst, const double* raw, const double* wtot,
                                 const double* csum, double lam, double beta, double* eout, hipStream_t st)
{
    (void)hipGetLastError();   // drop stale errors of earlier calls
    const int n = n_inst * R;
    energy_combine_kernel<<<(n + 255) / 256, 256, 0, st>>>(kind, R, q, n_inst, raw, wtot, csum, lam, beta, eout);
    return hipGetLastError();
}

hipError_t launch_colsum_combine(int R, int q, int n_inst, const long long* fx, double scale, double* csum,
                                 double* ctil, hipStream_t st)
{
    (void)hipGetLastError();   // drop stale errors of earlier calls
    const int n = n_inst * R;
    colsum_combine_kernel<<<(n + 255) / 256, 256, 0, st>>>(R, q, n_inst, fx, scale, csum, ctil);
    return hipGetLastError();
}

hipError_t launch_round(int kind, int32_t n, int32_t R, int32_t q, const float* h, int64_t srow, uint8_t* sigma,
                        hipStream_t st)
{
    (void)hipGetLastError();   // drop stale errors of earlier calls
    const size_t count = (size_t)n * R;
    if (count == 0) return hipSuccess;
    round_kernel<<<grid_for(count), 256, 0, st>>>(kind, n, R, q, h, srow, sigma);
    return hipGetLastError();
}

hipError_t launch_rows(int32_t n, int64_t w, float* dst, int64_t ds, const float* src, int64_t ss, float* z1,
                       float* z2, hipStream_t st)
{
    (void)hipGetLastError();   // drop stale errors of earlier calls
    const size_t count = (size_t)n * w;
    if (count == 0) return hipSuccess;
    auto al = [](const void* q) { return q == nullptr || (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
    if (w % 4 == 0 && ds % 4 == 0 && ss % 4 == 0 && al(dst) && al(src) && al(z1) && al(z2))
        rows_kernel<float4><<<grid_for(count / 4), 256, 0, st>>>(n, w, dst, ds, src, ss, z1, z2);
    else
        rows_kernel<float><<<grid_for(count), 256, 0, st>>>(n, w, dst, ds, src, ss, z1, z2);
    return hipGetLastError();
}

hipError_t launch_transpose_sigma(int32_t n, int32_t R, const int32_t* sig_rn, uint8_t* sig_nr, hipStream_t st)
{
    (void)hipGetLastError();   // drop stale errors of earlier calls
    const size_t count = (size_t)n * R;
    if (count == 0) return hipSuccess;
    transpose_sigma_kernel<<<grid_for(count), 256, 0, st>>>(n, R, sig_rn, sig_nr);
    return hipGetLastError();
}

hipError_t launch_eval(const Problem& p, const LaunchGeom& geo, int waves, const Tile* tiles, int32_t R,
                       const uint8_t* sigma, double* vpart, int* spart, hipStream_t st)
{
    (void)hipGetLastError();   // drop stale errors of earlier calls
    dim3 g(geo.n_tiles, geo.nseg), b(64 * waves);
    int lanes_log2 = 0;
    while ((1 << lanes_log2) < geo.lanes) ++lanes_log2;
    const int L = geo.lanes;
    if (p.kind == KIND_MAXSAT) {
        const size_t lds = lds_bytes(waves, L, 1);
        if (p.sat_width == 2)
            eval_sat_kernel<2><<<g, b, lds, st>>>(p.row_off, (const void*)p.inc2, tiles, R, lanes_log2, sigma, vpart);
        else
            eval_sat_kernel<3><<<g, b, lds, st>>>(p.row_off, (const void*)p.inc4, tiles, R, lanes_log2, sigma, vpart);
    } else if (p.kind == KIND_MAXCUT && R % 4 == 0 && (reinterpret_cast<uintptr_t>(sigma) & 3) == 0) {
        const LaunchGeom g4 = make_geom(4, R, waves);
        int l4 = 0;
        while ((1 << l4) < g4.lanes) ++l4;
        eval_cut4_kernel<<<dim3(geo.n_tiles, g4.nseg), b, lds_bytes(waves, g4.lanes, 4), st>>>(
            p.row_off, p.adj, tiles, R, l4, sigma, vpart);
    } else if (p.kind == KIND_MAXCUT) {
        eval_graph_kernel<1><<<g, b, lds_bytes(waves, L, 1), st>>>(p.row_off, p.adj, nullptr, tiles, R, lanes_log2,
                                                                    sigma, vpart, spart);
    } else {
        const size_t lds = lds_bytes(waves, L, p.q);
        switch (p.q) {
        case 2: eval_graph_kernel<2><<<g, b, lds, st>>>(p.row_off, p.adj, p.nw, tiles, R, lanes_log2, sigma, vpart, spart); break;
        case 4: eval_graph_kernel<4><<<g, b, lds, st>>>(p.row_off, p.adj, p.nw, tiles, R, lanes_log2, sigma, vpart, spart); break;
        case 8: eval_graph_kernel<8><<<g, b, lds, st>>>(p.row_off, p.adj, p.nw, tiles, R, lanes_log2, sigma, vpart, spart); break;
        case 16: eval_graph_kernel<16><<<g, b, lds, st>>>(p.row_off, p.adj, p.nw, tiles, R, lanes_log2, sigma, vpart, spart); break;
        case 32: eval_graph_kernel<32><<<g, b, lds, st>>>(p.row_off, p.adj, p.nw, tiles, R, lanes_log2, sigma, vpart, spart); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_sizes_widen(size_t count, const int* in, long long* out, hipStream_t st)
{
    (void)hipGetLastError();   // drop stale errors of earlier calls
    if (count == 0) return hipSuccess;
    sizes_widen_kernel<<<grid_for(count), 256, 0, st>>>(count, in, out);
    return hipGetLastError();
}

hipError_t launch_best_update(int kind, int R, int n_inst, int q, double lam, const double* vout,
                              const long long* sout, const double* v2, double* best, hipStream_t st)
{
    (void)hipGetLastError();   // drop stale errors of earlier calls
    if (kind == KIND_BMINCUT && !v2) return hipErrorInvalidValue;
    const int n = n_inst * R;
    best_update_kernel<<<(n + 255) / 256, 256, 0, st>>>(kind, R, n_inst, q, lam, vout, sout, v2, best);
    return hipGetLastError();
}

}  // namespace fem
