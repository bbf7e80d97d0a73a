// Internal declarations of the FEM library (host structures, kernel launch
// parameters).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace fem {

enum Kind { KIND_MAXCUT = 0, KIND_BMINCUT = 1, KIND_MAXSAT = 2 };

// One tile = a contiguous row range of a single instance; one workgroup per
// tile (times the replica segments along grid.y).
struct Tile {
    int32_t inst, row_begin, row_end, slot;   // slot: index of the tile's partial sums
};

// Device-resident problem.
struct Problem {
    int device = 0;
    int kind = KIND_MAXCUT;
    int32_t n = 0;         // total rows (nodes / variables) over all instances
    int32_t q = 2;         // states (2 for one-logit kinds)
    int64_t nnz = 0;       // adjacency entries or literal incidences
    int32_t n_inst = 1;
    int32_t sat_width = 2; // Max-k-SAT: other literals stored per incidence (2 or 3)
    int64_t n_clauses = 0;
    bool integral = true;  // all weights integral (exact integer cut values)
    std::vector<int32_t> inst_off;   // host [n_inst+1] node offsets
    std::vector<double> inst_wtot;   // host [n_inst] sum of undirected weights
    // device arrays
    int64_t* row_off = nullptr;      // [n+1]
    int2* adj = nullptr;             // graphs: {col, float bits of w}
    int32_t* adj_pm1 = nullptr;      // MaxCut with every weight +-1: col | (w < 0) << 31 (4 B per entry)
    int2* inc2 = nullptr;            // Max-k-SAT, <= 2 other literals per incidence
    int4* inc4 = nullptr;            // Max-k-SAT, <= 3 other literals per incidence
    float* wdeg = nullptr;           // bMinCut: sum_j W_ij per node
    double* nrm = nullptr;           // graphs: sum_j |W_ij| per node (normalisers of the manipulated gradients)
    int32_t* nw = nullptr;           // bMinCut node weights V_i (null: all 1)
    double* v2 = nullptr;            // bMinCut: [n_inst] sum_i V_i^2 per instance
    int32_t* inst_off_d = nullptr;   // [n_inst+1] node offsets of the instances
    // dense MaxCut: W as a zero-padded row-major float matrix [dense_ld][dense_ld]
    // (the CSR above is still built, for read-out and evaluation)
    float* dense_w = nullptr;
    int32_t dense_ld = 0;
    int8_t* dense_w8 = nullptr;      // the same as int8 when W is integral with |W| <= 127
    // host copies kept for batching and validation
    std::vector<int64_t> h_row_off;
    std::vector<int2> h_adj;
    std::vector<int2> h_inc2;
    std::vector<int4> h_inc4;
    std::vector<float> h_wdeg;
    std::vector<double> h_nrm;
    std::vector<int32_t> h_nw;       // empty: unit node weights
    std::vector<double> inst_v2;     // host [n_inst] sum_i V_i^2 (the node count for unit weights)
};

// Marginal-copy literal packing for Max-k-SAT incidence records:
//   bit 31: literal is positive; bits 0..29: variable; the value
//   SAT_NONE in bits 0..29 marks an unused slot (treated as a false literal
//   with probability 1, i.e. a neutral factor).
constexpr uint32_t SAT_VAR_MASK = 0x3FFFFFFFu;
constexpr uint32_t SAT_NONE = 0x3FFFFFFFu;
constexpr uint32_t SAT_POS = 0x80000000u;
// flag bits carried in bit 30 of the first / second slot
constexpr uint32_t SAT_FLAG = 0x40000000u;   // slot0: own literal positive; slot1: owner incidence

// Largest workgroup of a step kernel: register-heavy instantiations (8 values
// per lane; Potts with q >= 8) get a smaller bound so that the compiler may use
// up to 256 (512 threads) or 512 (256 threads) VGPRs without spilling.
__host__ __device__ constexpr int step_max_threads(int kind, int per_lane)
{
    return kind == KIND_BMINCUT ? (per_lane >= 16 ? 256 : (per_lane >= 8 ? 512 : 1024))
                                : (per_lane >= 8 ? 512 : 1024);
}

// bMinCut step kernel: per-lane running sums in LDS up to q = 16 (q + 3
// doubles per thread); the block reduction reuses that space
__host__ __device__ constexpr bool potts_lds_acc(int q) { return q <= 16; }
inline size_t potts_step_lds(int threads, int lanes, int q)
{
    const size_t red = (size_t)(threads / 64) * lanes * (q > 3 ? q : 3) * 8;
    const size_t acc = potts_lds_acc(q) ? (size_t)threads * (q + 3) * 8 : 0;
    return red > acc ? red : acc;
}

struct TileShape {
    int vec = 1, waves = 4, rows = 4;
    int nt = 0;      // non-temporal access to h, m1, m2
    int lanes = 0;   // cap on lanes per team (power of two <= 64; 0 = 64)
};

// Default launch shape before tuning: four waves, four rows per team, and as
// many replicas per lane as keep a team's row within one wave.
inline TileShape default_shape(int kind, int R)
{
    TileShape t;
    t.waves = 4;
    t.rows = 4;
    if (kind == KIND_BMINCUT) {
        t.vec = 1;
        return t;
    }
    if (R % 4 == 0 && R >= 128) t.vec = 4;
    else if (R % 2 == 0 && R >= 64) t.vec = 2;
    else t.vec = 1;
    return t;
}

// Per-step scalars, computed on the host in double and passed as float.
struct StepScalars {
    double inv_beta_d;   // 1/beta and lambda in double for the gradient combination
    double lam_d;
    double gamma_d;      // gamma_grad (manipulated gradients and Max-k-SAT; 1 otherwise)
    float inv_beta;
    float lam;
    float step_size;   // lr / (1 - b1^n)
    float bc2_sqrt;    // sqrt(1 - b2^n)
    float inv_bc2_sqrt;   // 1 / sqrt(1 - b2^n)
    float b1, one_m_b1, b2, one_m_b2, eps, wd;
    int opt;            // 0 Adam, 1 RMSprop, 2 SGD
    int first;          // SGD: first step (the momentum buffer starts as g)
    float mom, damp, rms_alpha, one_m_rms, lr;
};

struct LaunchGeom {
    int lanes;        // lanes per team (power of two, <= 64)
    int nseg;         // replica segments
    int teams_per_block;
    int n_tiles;
    int seg_major;    // grid (nseg, n_tiles) instead of (n_tiles, nseg)
};

inline int pow2ceil(int x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Teams of lanes covering R replicas at per_lane values per lane, at most
// max_lanes lanes (0 or 64: a full wave), and the replica segments left over.
inline LaunchGeom make_geom(int per_lane, int R, int waves, int max_lanes = 64)
{
    LaunchGeom g{};
    const int need = (R + per_lane - 1) / per_lane;
    const int cap = max_lanes > 0 ? max_lanes : 64;
    const int p2 = pow2ceil(need);
    g.lanes = cap < p2 ? cap : p2;
    g.nseg = (need + g.lanes - 1) / g.lanes;
    g.teams_per_block = waves * (64 / g.lanes);
    return g;
}

// Arguments shared by the step kernels.
struct StepArgs {
    const int64_t* row_off;
    const int2* adj;
    const int32_t* adj_pm1;       // the same entries in 4 bytes when every weight is +-1, else null
    const int2* inc2;
    const int4* inc4;
    const float* wdeg;
    const double* nrm;            // per-node sum_j |W_ij| (manipulated gradients)
    const int32_t* nw;            // bMinCut node weights (null: all 1)
    const Tile* tiles;
    const void* marg_cur;
    void* marg_nxt;
    float* h;                     // rows of h, m1, m2 are srow floats apart
    float* m1;
    float* m2;
    int64_t srow;
    float* grad;                  // may be null; [n][R(q)]
    double* epart;                // [n_tiles][NE][R] or null (no energies this step)
    const double* ctil;           // bMinCut: centred column sums C~ [inst][R][q]
    long long* cpart;             // bMinCut: column-sum partials of the new P [n_tiles][R][q]
    int32_t n;
    int32_t R;
    int32_t q;
    int32_t rw;                   // MaxCut manipulated: 32-bit words per row of the sign bits
    int32_t lanes_log2;
    int32_t seg_major;            // block -> (tile, segment) mapping of the grid
    StepScalars sc;
};

// record the text of a failure for fem_last_error() (fem_host.hip); returns st
int set_error(int st, const char* msg);

// host-side kernel launchers (fem_kernels.hip)
hipError_t launch_step(int kind, int dtype, int vec, bool nt, const LaunchGeom& g, int waves,
                       const StepArgs& a, hipStream_t st);
// marginal copy of a.h into a.marg_nxt (count = n*R values for one-logit kinds);
// for bMinCut also the column-sum partials a.cpart
hipError_t launch_init_marginals(int kind, int dtype, const LaunchGeom& g, int waves,
                                 const StepArgs& a, size_t count, hipStream_t st);
// out[inst][c] = sum over the instance's tiles of part[tile][c] (two fixed-order stages)
template <typename T>
hipError_t launch_seg_reduce(const T* part, int cols, const int32_t* chunk_off, int n_chunks,
                             const int32_t* inst_chunk_off, int n_inst, T* tmp, T* out,
                             hipStream_t st);
// the same energies from the per-tile partials in one launch (instances of
// few tiles): part [tile][NE][R], tiles of instance b from chunk
// inst_chunk_off[b] to inst_chunk_off[b + 1]
hipError_t launch_energy_finish(int kind, int R, int q, int NE, int n_inst, const double* part,
                                const int32_t* chunk_off, const int32_t* inst_chunk_off, const double* wtot,
                                const double* csum, double lam, double beta, double* eout, hipStream_t st);
hipError_t launch_energy_combine(int kind, int R, int q, int n_inst, const double* raw,
                                 const double* wtot, const double* csum, double lam, double beta,
                                 double* eout, hipStream_t st);
// manipulated gradients (fem_manip.hip): the step kernel, and the read-out copy
// of a.h (sign bits or argmax states, with per-tile state counts for bMinCut)
hipError_t launch_manip_step(int kind, int vec, bool nt, const LaunchGeom& g, int waves, const StepArgs& a,
                             hipStream_t st);
hipError_t launch_manip_init(int kind, const LaunchGeom& g, int waves, const StepArgs& a, hipStream_t st);
// csum = fx * scale (2^-40 for fixed-point marginal sums, 1 for state counts),
// ctil = csum minus its mean over the states
hipError_t launch_colsum_combine(int R, int q, int n_inst, const long long* fx, double scale, double* csum,
                                 double* ctil, hipStream_t st);
hipError_t launch_round(int kind, int32_t n, int32_t R, int32_t q, const float* h, int64_t srow, uint8_t* sigma,
                        hipStream_t st);
// n rows of w floats: dst[i ds + c] = src[i ss + c] (src not null), and zeros
// into z1[i ds + c] and z2[i ds + c] (where not null)
hipError_t launch_rows(int32_t n, int64_t w, float* dst, int64_t ds, const float* src, int64_t ss, float* z1,
                       float* z2, hipStream_t st);
hipError_t launch_transpose_sigma(int32_t n, int32_t R, const int32_t* sig_rn, uint8_t* sig_nr,
                                  hipStream_t st);
hipError_t launch_eval(const Problem& p, const LaunchGeom& g, int waves, const Tile* tiles,
                       int32_t R, const uint8_t* sigma, double* vpart, int* spart,
                       hipStream_t st);
hipError_t launch_sizes_widen(size_t count, const int* in, long long* out, hipStream_t st);
// v2: bMinCut per-instance sum_i V_i^2 (the constant that makes the balance
// penalty vanish on a perfect split of unit weights)
hipError_t launch_best_update(int kind, int R, int n_inst, int q, double lam, const double* vout,
                              const long long* sout, const double* v2, double* best, hipStream_t st);

}  // namespace fem

// Problems are reference counted: every solver holds one reference, so a
// problem released by its owner stays alive until its last solver is gone.
struct fem_problem {
    fem::Problem p;
    int refs = 0;
    bool released = false;
};
