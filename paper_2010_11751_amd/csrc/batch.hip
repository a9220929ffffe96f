// Batched ensemble of independent cavities (D3Q19, any storage type, 2Pop or
// AA). All cavities live in one pool; one kernel launch per time step covers
// every cavity through a (cavity, tile) table, each block reading its
// cavity's field description and relaxation rates. The step loop can be
// captured once in a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <string>
#include <vector>

#include "internal.hpp"
#include "lbm.h"

using namespace lbm;

namespace lbm_detail {
int set_error(int code, const std::string& msg);
}

namespace {

int fail(int code, const std::string& msg) { return lbm_detail::set_error(code, msg); }

int hip_fail(hipError_t e, const char* what)
{
    return fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                              \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

using LaunchFn = hipError_t (*)(const Launch&, hipStream_t);

LaunchFn pick_tu19(int dtype)
{
    return dtype == LBM_F64 ? launch_q19_f64 : dtype == LBM_F32_SHIFTED ? launch_q19_f32 : launch_q19_f16;
}

size_t elem_bytes(int dtype) { return dtype == LBM_F64 ? 8 : dtype == LBM_F32_SHIFTED ? 4 : 2; }
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
uint32_t grid_for(uint64_t n, int block) { return (uint32_t)((n + block - 1) / block); }

// Padding (elements) around each cavity's streams, covering the largest
// neighbour offset ny*nz + nz + 1 (the step kernels load speculatively).
size_t halo_of(const lbm_cavity_desc& d) { return align_up((size_t)d.ny * d.nz + d.nz + 1, 64); }

__global__ void kb_flag_types(uint8_t* fl, int nx, int ny, int nz)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t n = (uint32_t)nx * ny * nz;
    if (i >= n) return;
    const int z = (int)(i % nz), y = (int)((i / nz) % ny), x = (int)(i / ((uint32_t)ny * nz));
    const bool inside = x >= 1 && x <= nx - 2 && y >= 1 && y <= ny - 2 && z >= 1 && z <= nz - 2;
    fl[i] = inside ? FL_FLUID : (z == nz - 1 ? FL_LID : FL_WALL);
}

// Fast-path hints of a cavity's fluid cells (they never sit on a box face):
// the wall-plane code when the non-fluid neighbours are exactly the nine on
// one side (the cell is one layer inside a single face), NEARWALL along the
// edges and corners where two faces meet.
__global__ void kb_flag_hints(uint8_t* fl, int nx, int ny, int nz)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t n = (uint32_t)nx * ny * nz;
    if (i >= n || (fl[i] & FL_TYPE) != FL_FLUID) return;
    const int z = (int)(i % nz), y = (int)((i / nz) % ny), x = (int)(i / ((uint32_t)ny * nz));
    const int c[3] = {x, y, z}, hi[3] = {nx - 2, ny - 2, nz - 2};
    int planes = 0, code = 0;
    for (int a = 0; a < 3; ++a) {
        if (c[a] == 1) { ++planes; code = 1 + 2 * a; }
        if (c[a] == hi[a]) { ++planes; code = 2 + 2 * a; }
    }
    if (planes == 1) fl[i] |= (uint8_t)(code << FL_PLANE_SHIFT);
    else if (planes > 1) fl[i] |= FL_NEARWALL;
}

__global__ void kb_reduce_pairs(const double* partial, int nblocks, double* result)
{
    __shared__ double sm[2][256];
    double m = 0.0, e = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) {
        m += partial[2 * (size_t)b];
        e += partial[2 * (size_t)b + 1];
    }
    sm[0][threadIdx.x] = m;
    sm[1][threadIdx.x] = e;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sm[0][threadIdx.x] += sm[0][threadIdx.x + s];
            sm[1][threadIdx.x] += sm[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        result[0] = sm[0][0];
        result[1] = sm[1][0];
    }
}

}  // namespace

struct lbm_batch {
    int count = 0;
    int scheme = LBM_AA, collision = LBM_BGK, dtype = LBM_F64;
    lbm_batch_opts opts{};
    std::vector<lbm_cavity_desc> desc;
    std::vector<BatchCavity> cav[2];  // [0]: pop->out, [1]: out->pop (2Pop parity)
    BatchCavity* d_cav[2] = {nullptr, nullptr};
    uint32_t* d_tiles = nullptr;
    uint32_t ntiles = 0;
    void* pool = nullptr;
    uint8_t* flags = nullptr;
    double* partial = nullptr;
    size_t partial_len = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int block = 256;
    int elem = 8;                   // bytes per stored value
    bool no_residency_cap = false;  // LBM_NO_RESIDENCY_CAP set: every wave may be resident
    int64_t cells = 0, fluid = 0;
    int phase = 0;  // AA phase, or 2Pop parity (which array is current)
    hipGraphExec_t graph = nullptr;
    int graph_steps = 0;
    int graph_phase = -1;
    LaunchFn launch = nullptr;
};

namespace {

int build_tiles(lbm_batch* b, int block)
{
    std::vector<uint32_t> t;
    for (int c = 0; c < b->count; ++c) {
        const uint32_t n = b->cav[0][c].F.ntot;
        const uint32_t nt = grid_for(n, block);
        if (nt > 0xffffu) return fail(LBM_EUNSUPPORTED, "cavity too large for the tile table");
        for (uint32_t j = 0; j < nt; ++j) t.push_back(((uint32_t)c << 16) | j);
    }
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    b->d_tiles = nullptr;
    HIP_TRY(hipMalloc(&b->d_tiles, sizeof(uint32_t) * t.size()), "hipMalloc tiles");
    HIP_TRY(hipMemcpy(b->d_tiles, t.data(), sizeof(uint32_t) * t.size(), hipMemcpyHostToDevice), "hipMemcpy tiles");
    b->ntiles = (uint32_t)t.size();
    b->block = block;
    return LBM_OK;
}

int launch_batch_step(lbm_batch* b)
{
    Launch L{};
    L.op = OP_STEP_BATCH;
    L.model = b->collision;
    L.layout = LAYOUT_SOA;
    L.block = b->block;
    L.grid = b->ntiles;
    L.tiles = b->d_tiles;
    if (b->scheme == LBM_2POP) {
        L.kind = KIND_2POP;
        L.cav = b->d_cav[b->phase];
    } else {
        L.kind = b->phase ? KIND_AA_ODD : KIND_AA_EVEN;
        L.cav = b->d_cav[0];
    }
    L.lds = b->no_residency_cap ? 0 : residency_lds(step_waves(b->elem, L.kind), b->block);
    hipError_t e = b->launch(L, b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch step launch");
    b->phase ^= 1;
    return LBM_OK;
}

int init_batch_state(lbm_batch* b)
{
    for (int c = 0; c < b->count; ++c) {
        const BatchCavity& B = b->cav[0][c];
        Launch L{};
        L.op = OP_INIT;
        L.model = b->collision;
        L.layout = LAYOUT_SOA;
        L.block = 256;
        L.grid = grid_for(B.F.ntot, 256);
        L.F = B.F;
        L.init.lid[0] = b->desc[c].u_lid;
        hipError_t e = b->launch(L, b->stream);
        if (e != hipSuccess) return hip_fail(e, "batch init launch");
    }
    b->phase = 0;
    return LBM_OK;
}

// Field of cavity idx holding the current state, and its AA phase.
Field current_field(const lbm_batch* b, int idx, int* aa_odd)
{
    *aa_odd = b->scheme == LBM_AA ? b->phase : 0;
    Field F = b->cav[0][idx].F;
    if (b->scheme == LBM_2POP && b->phase) std::swap(F.pop, F.out);
    F.out = nullptr;
    return F;
}

int autotune_batch(lbm_batch* b)
{
    static const int cand[] = {64, 128, 256, 512, 1024};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
    float best = 1e30f;
    int best_b = 256;
    for (int c : cand) {
        if (c > max_step_block(19, b->collision, 8)) continue;
        int rc = build_tiles(b, c);
        for (int s = 0; !rc && s < 2; ++s) rc = launch_batch_step(b);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(e0, b->stream), "hipEventRecord");
        for (int s = 0; !rc && s < 6; ++s) rc = launch_batch_step(b);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(e1, b->stream), "hipEventRecord");
        HIP_TRY(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        if (ms < best) {
            best = ms;
            best_b = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return build_tiles(b, best_b);
}

// Key of an ensemble in the autotune cache: GPU architecture, scheme,
// collision, storage type, cavity count and an FNV-1a hash of the cavity sizes.
std::string cache_key(const lbm_batch* b)
{
    hipDeviceProp_t prop{};
    int dev = 0;
    std::string arch = "gpu";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        arch = arch.substr(0, arch.find(':'));
    }
    uint64_t h = 1469598103934665603ull;
    for (const lbm_cavity_desc& c : b->desc)
        for (int v : {c.nx, c.ny, c.nz}) {
            h ^= (uint64_t)(uint32_t)v;
            h *= 1099511628211ull;
        }
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s/q19/s%d/c%d/d%d/n%d/%016llx", arch.c_str(), b->scheme, b->collision, b->dtype,
                  b->count, (unsigned long long)h);
    return buf;
}

int cached_block(const char* path, const std::string& key)
{
    FILE* f = std::fopen(path, "r");
    if (!f) return 0;
    char k[256];
    int blk = 0, found = 0;
    while (std::fscanf(f, "%255s %d", k, &blk) == 2)
        if (key == k && blk >= 64 && blk <= 1024 && blk % 64 == 0) found = blk;
    std::fclose(f);
    return found;
}

void free_batch(lbm_batch* b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->d_cav[0]) (void)hipFree(b->d_cav[0]);
    if (b->d_cav[1]) (void)hipFree(b->d_cav[1]);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->pool) (void)hipFree(b->pool);
    if (b->flags) (void)hipFree(b->flags);
    if (b->partial) (void)hipFree(b->partial);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // namespace

extern "C" {

lbm_batch* lbm_batch_create(int count, const lbm_cavity_desc* d, int scheme, int collision, int storage_dtype,
                            const lbm_batch_opts* opts)
{
    if (count <= 0 || count > 0xffff || !d) {
        fail(LBM_EINVAL, "count must be in [1, 65535] with a description array");
        return nullptr;
    }
    if (scheme != LBM_2POP && scheme != LBM_AA) {
        fail(scheme == LBM_SWAP || scheme == LBM_2POP_PULL ? LBM_EUNSUPPORTED : LBM_EINVAL, "batch schemes: 2Pop or AA");
        return nullptr;
    }
    if (collision < LBM_BGK || collision > LBM_K || storage_dtype < LBM_F64 || storage_dtype > LBM_F16_SHIFTED) {
        fail(LBM_EINVAL, "unknown collision model or storage dtype");
        return nullptr;
    }
    for (int c = 0; c < count; ++c) {
        const lbm_cavity_desc& x = d[c];
        if (x.nx < 3 || x.ny < 3 || x.nz < 3 || (int64_t)x.nx * x.ny * x.nz > 0x7fffffffLL) {
            fail(LBM_EINVAL, "cavity " + std::to_string(c) + ": dimensions must be >= 3");
            return nullptr;
        }
        if (!(x.omega > 0.0 && x.omega < 2.0) || !(std::fabs(x.u_lid) < 0.4)) {
            fail(LBM_EINVAL, "cavity " + std::to_string(c) + ": omega in (0,2), |u_lid| < 0.4");
            return nullptr;
        }
    }
    lbm_batch* b = new lbm_batch();
    b->count = count;
    b->scheme = scheme;
    b->collision = collision;
    b->elem = storage_dtype == LBM_F64 ? 8 : storage_dtype == LBM_F32_SHIFTED ? 4 : 2;
    b->no_residency_cap = std::getenv("LBM_NO_RESIDENCY_CAP") != nullptr;
    b->dtype = storage_dtype;
    b->desc.assign(d, d + count);
    if (opts) b->opts = *opts;
    if (b->opts.graph_steps <= 0) b->opts.graph_steps = 100;
    if (b->opts.graph_steps % 2) ++b->opts.graph_steps;
    b->launch = pick_tu19(storage_dtype);
    auto bail = [&](int code) -> lbm_batch* {
        (void)code;
        free_batch(b);
        return nullptr;
    };
    if (b->opts.stream) {
        b->stream = (hipStream_t)b->opts.stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            hip_fail(e, "hipStreamCreate");
            return bail(0);
        }
        b->own_stream = true;
    }

    // Pool layout: per cavity Q*stride elements (x2 for 2Pop), 256-byte aligned.
    const size_t s = elem_bytes(storage_dtype);
    const int Q = 19;
    std::vector<size_t> off(count), foff(count);
    size_t total = 0, ftotal = 0;
    b->cav[0].resize(count);
    b->cav[1].resize(count);
    for (int c = 0; c < count; ++c) {
        const uint32_t n = (uint32_t)d[c].nx * d[c].ny * d[c].nz;
        const int64_t stride = (int64_t)align_up(n, 128);
        const size_t bytes = align_up(((size_t)Q * stride + 2 * halo_of(d[c])) * s, 256);
        off[c] = total;
        total += bytes * (scheme == LBM_2POP ? 2 : 1);
        foff[c] = ftotal;
        ftotal += align_up(n, 256);
        b->cells += n;
        b->fluid += (int64_t)(d[c].nx - 2) * (d[c].ny - 2) * (d[c].nz - 2);
        Field F{};
        F.stride = stride;
        F.ntot = n;
        F.nx = d[c].nx;
        F.ny = d[c].ny;
        F.nz = d[c].nz;
        RelaxD r{};
        r.omega = d[c].omega;
        const double lam = d[c].trt_lambda > 0.0 ? d[c].trt_lambda : 0.25;
        r.omega_m = collision == LBM_TRT ? 1.0 / (0.5 + lam / (1.0 / d[c].omega - 0.5)) : d[c].omega;
        r.omega_b = d[c].omega;
        r.omega3 = 1.0;
        r.omega4 = 1.0;
        b->cav[0][c] = BatchCavity{F, r};
    }
    hipError_t e = hipMalloc(&b->pool, total);
    if (e == hipSuccess) e = hipMalloc((void**)&b->flags, ftotal);
    if (e != hipSuccess) {
        hip_fail(e, "hipMalloc batch pool");
        return bail(0);
    }
    size_t maxblocks = 0;
    for (int c = 0; c < count; ++c) {
        BatchCavity& B = b->cav[0][c];
        const size_t bytes = align_up(((size_t)Q * B.F.stride + 2 * halo_of(d[c])) * s, 256);
        const size_t skip = halo_of(d[c]) * s;
        B.F.pop = (char*)b->pool + off[c] + skip;
        B.F.out = scheme == LBM_2POP ? (char*)b->pool + off[c] + bytes + skip : nullptr;
        B.F.flags = b->flags + foff[c];
        b->cav[1][c] = B;
        std::swap(b->cav[1][c].F.pop, b->cav[1][c].F.out);
        maxblocks = std::max<size_t>(maxblocks, grid_for(B.F.ntot, 256));
        const uint32_t g = grid_for(B.F.ntot, 256);
        kb_flag_types<<<g, 256, 0, b->stream>>>((uint8_t*)B.F.flags, B.F.nx, B.F.ny, B.F.nz);
        kb_flag_hints<<<g, 256, 0, b->stream>>>((uint8_t*)B.F.flags, B.F.nx, B.F.ny, B.F.nz);
    }
    b->partial_len = 2 * maxblocks + 2;
    e = hipMalloc((void**)&b->partial, sizeof(double) * b->partial_len);
    for (int p = 0; p < 2 && e == hipSuccess; ++p) {
        e = hipMalloc((void**)&b->d_cav[p], sizeof(BatchCavity) * count);
        if (e == hipSuccess)
            e = hipMemcpy(b->d_cav[p], b->cav[p].data(), sizeof(BatchCavity) * count, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        hip_fail(e, "batch tables");
        return bail(0);
    }
    if (init_batch_state(b)) return bail(0);
    int block = b->opts.block_size > 0 ? b->opts.block_size : 256;
    if (block % 64 || block > 1024) {
        fail(LBM_EINVAL, "block_size must be a multiple of 64 up to 1024");
        return bail(0);
    }
    if (build_tiles(b, std::min(block, max_step_block(19, b->collision, 8)))) return bail(0);
    if (b->opts.autotune) {
        const std::string key = b->opts.autotune_cache ? cache_key(b) : std::string();
        const int hit = b->opts.autotune_cache ? cached_block(b->opts.autotune_cache, key) : 0;
        if (hit && hit <= max_step_block(19, b->collision, 8)) {
            if (build_tiles(b, hit)) return bail(0);
        } else {
            if (autotune_batch(b) || init_batch_state(b)) return bail(0);
            if (b->opts.autotune_cache) {
                if (FILE* f = std::fopen(b->opts.autotune_cache, "a")) {
                    std::fprintf(f, "%s %d\n", key.c_str(), b->block);
                    std::fclose(f);
                }
            }
        }
    }
    b->opts.autotune_cache = nullptr;  // the caller's string is only read at creation
    e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        hip_fail(e, "batch initialisation");
        return bail(0);
    }
    return b;
}

void lbm_batch_destroy(lbm_batch* b) { free_batch(b); }

static int capture_graph(lbm_batch* b)
{
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    hipGraph_t g = nullptr;
    const int phase0 = b->phase;
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    int rc = LBM_OK;
    for (int s = 0; s < b->opts.graph_steps && !rc; ++s) rc = launch_batch_step(b);
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    b->phase = phase0;  // capture only recorded the launches
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    b->graph_steps = b->opts.graph_steps;
    b->graph_phase = phase0;
    return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int n)
{
    if (!b) return fail(LBM_EINVAL, "null batch");
    if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
    if (b->opts.use_graph) {
        while (n >= b->opts.graph_steps) {
            if (!b->graph || b->graph_phase != b->phase) {
                int rc = capture_graph(b);
                if (rc) return rc;
            }
            HIP_TRY(hipGraphLaunch(b->graph, b->stream), "hipGraphLaunch");
            n -= b->graph_steps;  // graph_steps is even: the phase is unchanged
        }
    }
    for (int s = 0; s < n; ++s) {
        int rc = launch_batch_step(b);
        if (rc) return rc;
    }
    return LBM_OK;
}

int lbm_batch_step_sequential(lbm_batch* b, int n)
{
    if (!b) return fail(LBM_EINVAL, "null batch");
    if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
    for (int s = 0; s < n; ++s) {
        for (int c = 0; c < b->count; ++c) {
            Launch L{};
            L.op = OP_STEP_ALL;
            L.model = b->collision;
            L.layout = LAYOUT_SOA;
            L.block = b->block;
            L.grid = grid_for(b->cav[0][c].F.ntot, b->block);
            L.F = b->cav[b->scheme == LBM_2POP ? b->phase : 0][c].F;
            L.relax = b->cav[0][c].relax;
            L.kind = b->scheme == LBM_2POP ? KIND_2POP : (b->phase ? KIND_AA_ODD : KIND_AA_EVEN);
            hipError_t e = b->launch(L, b->stream);
            if (e != hipSuccess) return hip_fail(e, "sequential step launch");
        }
        b->phase ^= 1;
    }
    return LBM_OK;
}

int lbm_batch_macroscopic(lbm_batch* b, int idx, double* rho, double* u)
{
    if (!b || idx < 0 || idx >= b->count || !rho || !u) return fail(LBM_EINVAL, "bad argument");
    Launch L{};
    L.op = OP_MACRO;
    L.model = b->collision;
    L.layout = LAYOUT_SOA;
    L.F = current_field(b, idx, &L.aa_odd);
    L.block = 256;
    L.grid = grid_for(L.F.ntot, 256);
    L.d0 = rho;
    L.d1 = u;
    hipError_t e = b->launch(L, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch macroscopic");
    return LBM_OK;
}

int lbm_batch_get_populations(lbm_batch* b, int idx, double* f)
{
    if (!b || idx < 0 || idx >= b->count || !f) return fail(LBM_EINVAL, "bad argument");
    Launch L{};
    L.op = OP_GET;
    L.model = b->collision;
    L.layout = LAYOUT_SOA;
    L.F = current_field(b, idx, &L.aa_odd);
    L.block = 256;
    L.grid = grid_for(L.F.ntot, 256);
    L.d0 = f;
    hipError_t e = b->launch(L, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch populations");
    return LBM_OK;
}

int lbm_batch_invariants(lbm_batch* b, double* mass, double* kinetic_energy)
{
    if (!b || !mass || !kinetic_energy) return fail(LBM_EINVAL, "bad argument");
    for (int c = 0; c < b->count; ++c) {
        Launch L{};
        L.op = OP_INVARIANTS;
        L.model = b->collision;
        L.layout = LAYOUT_SOA;
        L.F = current_field(b, c, &L.aa_odd);
        L.block = 256;
        L.grid = grid_for(L.F.ntot, 256);
        L.d0 = b->partial;
        hipError_t e = b->launch(L, b->stream);
        if (e != hipSuccess) return hip_fail(e, "batch invariants");
        double* res = b->partial + b->partial_len - 2;
        kb_reduce_pairs<<<1, 256, 0, b->stream>>>(b->partial, (int)L.grid, res);
        double hr[2];
        HIP_TRY(hipMemcpyAsync(hr, res, sizeof(hr), hipMemcpyDeviceToHost, b->stream), "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
        mass[c] = hr[0];
        kinetic_energy[c] = hr[1];
    }
    return LBM_OK;
}

int lbm_batch_info(lbm_batch* b, int64_t* cells, int64_t* fluid_cells, int* block_size)
{
    if (!b) return fail(LBM_EINVAL, "null batch");
    if (cells) *cells = b->cells;
    if (fluid_cells) *fluid_cells = b->fluid;
    if (block_size) *block_size = b->block;
    return LBM_OK;
}

int lbm_batch_sync(lbm_batch* b)
{
    if (!b) return fail(LBM_EINVAL, "null batch");
    HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    return LBM_OK;
}

}  // extern "C"
