// Integer evaluation without device allocation (fem_eval_int_noalloc).
//
// fem_eval_int creates a solver for its per-tile partial sums, byte
// configurations and tile lists, and copies through host memory.  Callers that
// cannot allocate device memory (work recorded into a HIP graph, serving loops,
// harnesses that forbid hipMalloc) get the same evaluation from device-resident
// configurations, with every intermediate in one fixed per-device array,
// `scratch`, that lives as long as the process.  The work is the same as
// fem_eval_int's: the same tiles (rows per tile from the default launch shape,
// chunks of 64 tiles per instance), the same evaluation and reduction kernels,
// so the results are bit-identical to it.
//
// Host code never passes the array's name to a kernel: on the host that name
// is a stand-in, not a device address.  The device address is looked up once
// per device with hipGetSymbolAddress and kept.
#include "fem_dense.h"
#include "fem_device.h"
#include "fem_internal.h"
#include "../../include/fem.h"

#include <mutex>

namespace fem {

constexpr size_t NOALLOC_SCRATCH = (size_t)FEM_NOALLOC_SCRATCH_BYTES;
constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES];

// Device address of `scratch` on `device` (which must be current): looked up on
// the first call for that device, then reused.
static int scratch_address(int device, unsigned char** out)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES)
        return set_error(FEM_E_UNSUPPORTED, "device ordinal out of the supported range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            std::string msg = "hipGetSymbolAddress(scratch): ";
            msg += hipGetErrorString(e);
            return set_error(FEM_E_HIP, msg.c_str());
        }
        g_scratch_ptr[device] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[device]);
    return FEM_OK;
}

// ------------------------------------------------------------------ kernels
__global__ void noalloc_clear_kernel(int* __restrict__ p, int n)
{
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) p[k] = 0;
}

// Per-instance tile and chunk offsets: instance b holds ceil(rows_b / tile_rows)
// tiles and ceil(tiles_b / 64) chunks; exclusive prefix sums over b (one
// workgroup of 1024 threads, instances in rounds of 1024).
__global__ void __launch_bounds__(1024) noalloc_inst_offsets_kernel(const int32_t* __restrict__ inst_off, int n_inst,
                                                                    int tile_rows, int32_t* __restrict__ inst_tile_off,
                                                                    int32_t* __restrict__ inst_chunk_off)
{
    __shared__ int32_t st[1024], sc[1024];
    __shared__ int32_t carry_t, carry_c;
    const int tid = threadIdx.x;
    if (tid == 0) {
        carry_t = 0;
        carry_c = 0;
    }
    __syncthreads();
    for (int b0 = 0; b0 < n_inst; b0 += 1024) {
        const int b = b0 + tid;
        int32_t nt = 0, nc = 0;
        if (b < n_inst) {
            const int32_t rows = inst_off[b + 1] - inst_off[b];
            nt = (rows + tile_rows - 1) / tile_rows;
            nc = (nt + 63) / 64;
        }
        st[tid] = nt;
        sc[tid] = nc;
        __syncthreads();
        // inclusive Hillis-Steele scan
        for (int d = 1; d < 1024; d <<= 1) {
            const int32_t at = tid >= d ? st[tid - d] : 0;
            const int32_t ac = tid >= d ? sc[tid - d] : 0;
            __syncthreads();
            st[tid] += at;
            sc[tid] += ac;
            __syncthreads();
        }
        if (b < n_inst) {
            inst_tile_off[b] = carry_t + st[tid] - nt;
            inst_chunk_off[b] = carry_c + sc[tid] - nc;
        }
        __syncthreads();
        if (tid == 1023) {
            carry_t += st[1023];
            carry_c += sc[1023];
        }
        __syncthreads();
    }
    if (tid == 0) {
        inst_tile_off[n_inst] = carry_t;
        inst_chunk_off[n_inst] = carry_c;
    }
}

// last b in [0, n) with off[b] <= k (off nondecreasing, off[0] = 0 <= k)
__device__ __forceinline__ int last_at_most(const int32_t* __restrict__ off, int n, int32_t k)
{
    int lo = 0, hi = n;   // off[lo] <= k; answer in [lo, hi)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= k) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The tile list (natural order, slot = index) and the chunk offsets, as the
// solver builds them: chunk c of instance b starts at tile
// inst_tile_off[b] + 64 (c - inst_chunk_off[b]); chunk_off[n_chunks] = n_tiles.
__global__ void noalloc_tiles_kernel(const int32_t* __restrict__ inst_off, const int32_t* __restrict__ inst_tile_off,
                                     const int32_t* __restrict__ inst_chunk_off, int n_inst, int tile_rows,
                                     int n_tiles, int n_chunks, Tile* __restrict__ tiles,
                                     int32_t* __restrict__ chunk_off)
{
    const int total = n_tiles + n_chunks + 1;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < total; k += gridDim.x * blockDim.x) {
        if (k < n_tiles) {
            const int b = last_at_most(inst_tile_off, n_inst, k);
            const int32_t r0 = inst_off[b] + (k - inst_tile_off[b]) * tile_rows;
            const int32_t r1 = min(inst_off[b + 1], r0 + tile_rows);
            tiles[k] = Tile{b, r0, r1, k};
        } else if (k < n_tiles + n_chunks) {
            const int c = k - n_tiles;
            const int b = last_at_most(inst_chunk_off, n_inst, c);
            chunk_off[c] = inst_tile_off[b] + 64 * (c - inst_chunk_off[b]);
        } else {
            chunk_off[n_chunks] = n_tiles;
        }
    }
}

// int32 [R][n] configurations -> bytes [n][R]; bad[r] = 1 when replica r holds
// a state outside [0, q) (its byte is then written as 0)
__global__ void noalloc_sigma_kernel(int32_t n, int32_t R, int32_t q, const int32_t* __restrict__ in,
                                     uint8_t* __restrict__ out, int* __restrict__ bad)
{
    const size_t count = (size_t)n * R;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (size_t)gridDim.x * blockDim.x) {
        const size_t i = k / R, r = k % R;
        const int32_t v = in[r * (size_t)n + i];
        const bool ok = v >= 0 && v < q;
        if (!ok) atomicOr(bad + r, 1);
        out[k] = (uint8_t)(ok ? v : 0);
    }
}

// value[b][r]: the cut (ordered sum halved, rounded) or the number of
// unsatisfied clauses; sizes[b][r][s] widened; INT64_MIN and -1 for replicas
// whose configuration held an invalid state
__global__ void noalloc_finish_kernel(int kind, int n_inst, int32_t R, int32_t q, const double* __restrict__ vout,
                                      const int* __restrict__ sint, const int* __restrict__ bad,
                                      int64_t* __restrict__ value, int64_t* __restrict__ sizes)
{
    const size_t nv = (size_t)n_inst * R;
    const size_t ns = sizes ? nv * q : 0;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < nv + ns; k += (size_t)gridDim.x * blockDim.x) {
        if (k < nv) {
            const double v = vout[k];
            const int64_t x = kind == KIND_MAXSAT ? (int64_t)v : (int64_t)llround(0.5 * v);
            value[k] = bad[k % R] ? INT64_MIN : x;
        } else {
            const size_t j = k - nv;
            const size_t r = (j / q) % R;
            sizes[j] = bad[r] ? -1 : (int64_t)sint[j];
        }
    }
}

static unsigned grid_of(size_t count)
{
    const size_t g = (count + 255) / 256;
    return (unsigned)(g < 4096 ? (g ? g : 1) : 4096);
}

}  // namespace fem

using namespace fem;

extern "C" fem_status fem_eval_int_noalloc(const fem_problem* fp, int32_t R, const int32_t* sigma, int64_t* value,
                                           int64_t* sizes, void* hip_stream)
{
    if (!fp || !sigma || !value) return (fem_status)set_error(FEM_E_INVAL, "NULL argument");
    if (R < 1) return (fem_status)set_error(FEM_E_INVAL, "R must be >= 1");
    const Problem& p = fp->p;
    if (sizes && p.kind != KIND_BMINCUT) sizes = nullptr;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (hipSetDevice(p.device) != hipSuccess) return (fem_status)set_error(FEM_E_HIP, "hipSetDevice failed");

    // the tiling fem_eval_int uses: the default launch shape's rows per tile
    const TileShape shape = default_shape(p.kind, R);
    const LaunchGeom geo = make_geom(p.kind == KIND_BMINCUT ? 1 : shape.vec, R, shape.waves);
    const int tile_rows = p.dense_w ? DENSE_ROWS : geo.teams_per_block * shape.rows;
    size_t n_tiles = 0, n_chunks = 0;
    for (int b = 0; b < p.n_inst; ++b) {
        const size_t rows = (size_t)(p.inst_off[(size_t)b + 1] - p.inst_off[(size_t)b]);
        const size_t t = (rows + tile_rows - 1) / tile_rows;
        n_tiles += t;
        n_chunks += (t + 63) / 64;
    }
    LaunchGeom egeo = make_geom(1, R, shape.waves);
    if (n_tiles > (size_t)INT32_MAX / 2 || (size_t)egeo.nseg > 65535)
        return (fem_status)set_error(FEM_E_UNSUPPORTED, "problem too large for the allocation-free evaluation");
    egeo.n_tiles = (int)n_tiles;

    // scratch layout, each part aligned to 256 bytes
    const size_t Rz = (size_t)R, B = (size_t)p.n_inst, Q = (size_t)p.q;
    const bool bm = p.kind == KIND_BMINCUT;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) & ~(size_t)255;
        return at;
    };
    const size_t o_bad = take(Rz * 4);
    const size_t o_itile = take((B + 1) * 4);
    const size_t o_ichunk = take((B + 1) * 4);
    const size_t o_chunk = take((n_chunks + 1) * 4);
    const size_t o_tiles = take(n_tiles * sizeof(Tile));
    const size_t o_sig = take((size_t)p.n * Rz);
    const size_t o_vpart = take(n_tiles * Rz * 8);
    const size_t o_vtmp = take(n_chunks * Rz * 8);
    const size_t o_vout = take(B * Rz * 8);
    const size_t o_spart = bm ? take(n_tiles * Rz * Q * 4) : 0;
    const size_t o_stmp = bm ? take(n_chunks * Rz * Q * 4) : 0;
    const size_t o_sint = bm ? take(B * Rz * Q * 4) : 0;
    if (off > NOALLOC_SCRATCH) {
        char msg[200];
        snprintf(msg, sizeof msg,
                 "the allocation-free evaluation needs %zu bytes of scratch for n = %d, R = %d; its maximum is %zu",
                 off, p.n, R, NOALLOC_SCRATCH);
        return (fem_status)set_error(FEM_E_UNSUPPORTED, msg);
    }
    unsigned char* base = nullptr;
    {
        const int rc = scratch_address(p.device, &base);
        if (rc != FEM_OK) return (fem_status)rc;
    }
    int* bad = reinterpret_cast<int*>(base + o_bad);
    int32_t* itile = reinterpret_cast<int32_t*>(base + o_itile);
    int32_t* ichunk = reinterpret_cast<int32_t*>(base + o_ichunk);
    int32_t* chunk = reinterpret_cast<int32_t*>(base + o_chunk);
    Tile* tiles = reinterpret_cast<Tile*>(base + o_tiles);
    uint8_t* sig8 = base + o_sig;
    double* vpart = reinterpret_cast<double*>(base + o_vpart);
    double* vtmp = reinterpret_cast<double*>(base + o_vtmp);
    double* vout = reinterpret_cast<double*>(base + o_vout);
    int* spart = bm ? reinterpret_cast<int*>(base + o_spart) : nullptr;
    int* stmp = bm ? reinterpret_cast<int*>(base + o_stmp) : nullptr;
    int* sint = bm ? reinterpret_cast<int*>(base + o_sint) : nullptr;

    (void)hipGetLastError();   // drop stale errors of earlier calls
    noalloc_clear_kernel<<<grid_of(Rz), 256, 0, st>>>(bad, R);
    noalloc_inst_offsets_kernel<<<1, 1024, 0, st>>>(p.inst_off_d, p.n_inst, tile_rows, itile, ichunk);
    noalloc_tiles_kernel<<<grid_of(n_tiles + n_chunks + 1), 256, 0, st>>>(
        p.inst_off_d, itile, ichunk, p.n_inst, tile_rows, (int)n_tiles, (int)n_chunks, tiles, chunk);
    noalloc_sigma_kernel<<<grid_of((size_t)p.n * Rz), 256, 0, st>>>(p.n, R, p.q, sigma, sig8, bad);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_eval(p, egeo, shape.waves, tiles, R, sig8, vpart, spart, st);
    if (e == hipSuccess) e = launch_seg_reduce<double>(vpart, R, chunk, (int)n_chunks, ichunk, p.n_inst, vtmp, vout, st);
    if (e == hipSuccess && bm)
        e = launch_seg_reduce<int>(spart, R * p.q, chunk, (int)n_chunks, ichunk, p.n_inst, stmp, sint, st);
    if (e == hipSuccess) {
        noalloc_finish_kernel<<<grid_of(B * Rz * (sizes ? Q + 1 : 1)), 256, 0, st>>>(p.kind, p.n_inst, R, p.q, vout,
                                                                                    sint, bad, value, sizes);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        std::string msg = "allocation-free evaluation: ";
        msg += hipGetErrorString(e);
        return (fem_status)set_error(FEM_E_HIP, msg.c_str());
    }
    return FEM_OK;
}
