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
    std::vector<BatchCavity> cav[2];  // [0]: pop->out, [1]: out->pop (2Pop and pull: current array)
    BatchCavity* d_cav[2] = {nullptr, nullptr};
    std::vector<int> order;         // cavities by decreasing cell count (tile order)
    uint32_t* d_tiles = nullptr;
    uint32_t ntiles = 0;
    uint32_t* d_slow = nullptr;     // edge cells of every cavity, each cavity padded to whole waves
    uint32_t* d_wave_cav = nullptr; // cavity of each wave of d_slow
    uint32_t n_slow = 0;            // entries of d_slow, padding included
    int64_t n_edge = 0;             // edge cells
    void* pool = nullptr;
    uint8_t* flags = nullptr;
    double* partial = nullptr;
    size_t partial_len = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t aux = nullptr;      // runs the edge cells beside the fast part
    hipEvent_t fork = nullptr, join = nullptr;
    int block = 256;
    int cpt = 1;                    // runs of `block` cells per tile
    int waves = -1;                 // resident waves per SIMD of the fast kernel (-1: by kind, 0: no cap)
    int xcd = 1;                    // tile table dealt to the XCDs in contiguous parts
    int elem = 8;                   // bytes per stored value
    bool box = false;               // AA / pull on cavities below 2^24 cells: position-driven kernel
    bool no_residency_cap = false;  // LBM_NO_RESIDENCY_CAP set: every wave may be resident
    int64_t cells = 0, fluid = 0;
    int phase = 0;  // AA: parity of the next step; 2Pop pull: state is post-collision
    int cur = 0;    // 2Pop, 2Pop pull: index of the array holding the state
    hipGraphExec_t graph = nullptr;
    int graph_steps = 0;
    int graph_phase = -1, graph_cur = -1;
    LaunchFn launch = nullptr;
};

namespace {

int build_tiles(lbm_batch* b, int block, int cpt)
{
    std::vector<uint32_t> t;
    const uint64_t span_cells = (uint64_t)block * cpt;
    for (int c : b->order) {
        const Field& F = b->cav[0][c].F;
        const uint64_t span = (uint64_t)F.ntot - 2ull * (uint64_t)F.ny * F.nz;  // layers x = 1 .. nx-2
        const uint64_t nt = (span + span_cells - 1) / span_cells;
        if (nt > 0xffffu) return fail(LBM_EUNSUPPORTED, "cavity too large for the tile table");
        for (uint32_t j = 0; j < nt; ++j) t.push_back(((uint32_t)c << 16) | j);
    }
    while (t.size() % 8) t.push_back(0xffffffffu);  // the XCD split deals eight equal parts
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    b->d_tiles = nullptr;
    b->ntiles = (uint32_t)t.size();
    b->block = block;
    b->cpt = cpt;
    if (t.empty()) return LBM_OK;
    HIP_TRY(hipMalloc(&b->d_tiles, sizeof(uint32_t) * t.size()), "hipMalloc tiles");
    HIP_TRY(hipMemcpy(b->d_tiles, t.data(), sizeof(uint32_t) * t.size(), hipMemcpyHostToDevice), "hipMemcpy tiles");
    return LBM_OK;
}

// Edge-cell list: the fluid cells whose flags send them off the fast path
// (next to two or more walls), read back from the flags the device built.
int build_slow_list(lbm_batch* b, size_t flag_bytes)
{
    std::vector<uint8_t> fl(flag_bytes);
    HIP_TRY(hipMemcpy(fl.data(), b->flags, flag_bytes, hipMemcpyDeviceToHost), "hipMemcpy flags");
    std::vector<uint32_t> list, wave_cav;
    for (int c : b->order) {
        const Field& F = b->cav[0][c].F;
        const uint8_t* f = fl.data() + (F.flags - b->flags);
        const size_t first = list.size();
        for (uint32_t i = 0; i < F.ntot; ++i)
            if ((f[i] & FL_TYPE) == FL_FLUID && (f[i] & FL_SLOW)) list.push_back(i);
        b->n_edge += (int64_t)(list.size() - first);
        while ((list.size() - first) % 64) list.push_back(0xffffffffu);
        for (size_t w = first / 64; w < list.size() / 64; ++w) wave_cav.push_back((uint32_t)c);
    }
    b->n_slow = (uint32_t)list.size();
    if (list.empty()) return LBM_OK;
    HIP_TRY(hipMalloc(&b->d_slow, sizeof(uint32_t) * list.size()), "hipMalloc edge list");
    HIP_TRY(hipMalloc(&b->d_wave_cav, sizeof(uint32_t) * wave_cav.size()), "hipMalloc edge list");
    HIP_TRY(hipMemcpy(b->d_slow, list.data(), sizeof(uint32_t) * list.size(), hipMemcpyHostToDevice), "hipMemcpy");
    HIP_TRY(hipMemcpy(b->d_wave_cav, wave_cav.data(), sizeof(uint32_t) * wave_cav.size(), hipMemcpyHostToDevice),
            "hipMemcpy");
    return LBM_OK;
}

bool needs_edge_part(int kind) { return kind == KIND_2POP || kind == KIND_AA_ODD || kind == KIND_PULL; }

// The kind of the next step and the cavity table it runs on; advances the
// scheme's bookkeeping (AA parity, 2Pop array, pull state).
int next_step(lbm_batch* b, const BatchCavity** table)
{
    int kind;
    if (b->scheme == LBM_AA) {
        kind = b->phase ? KIND_AA_ODD : KIND_AA_EVEN;
        *table = b->d_cav[0];
        b->phase ^= 1;
    } else if (b->scheme == LBM_2POP) {
        kind = KIND_2POP;
        *table = b->d_cav[b->cur];
        b->cur ^= 1;
    } else if (!b->phase) {  // 2Pop pull from a pre-collision state: an AA even step in place
        kind = KIND_AA_EVEN;
        *table = b->d_cav[b->cur];
        b->phase = 1;
    } else {
        kind = KIND_PULL;
        *table = b->d_cav[b->cur];
        b->cur ^= 1;
    }
    return kind;
}

uint32_t batch_lds(const lbm_batch* b, int kind)
{
    if (b->no_residency_cap || b->waves == 0) return 0;
    return residency_lds(b->waves > 0 ? b->waves : step_waves(b->elem, kind), b->block);
}

// One time step of every cavity: the fast kernel over the tile table and,
// for the kinds that reach neighbours, the edge-cell kernel on the second
// stream (each cell owns the memory it reads and writes, so the two parts
// run concurrently; the main stream waits for both before the next step).
int launch_batch_step(lbm_batch* b)
{
    Launch L{};
    L.op = OP_STEP_BATCH;
    L.model = b->collision;
    L.layout = LAYOUT_SOA;
    L.kind = next_step(b, &L.cav);
    L.block = b->block;
    L.grid = b->ntiles;
    L.tiles = b->d_tiles;
    L.cpt = (uint32_t)b->cpt;
    L.lds = batch_lds(b, L.kind);
    L.box = b->box ? 1 : 0;
    L.xcd = (uint32_t)b->xcd;
    const bool edge = !b->box && needs_edge_part(L.kind) && b->n_slow > 0;
    if (edge) {
        HIP_TRY(hipEventRecord(b->fork, b->stream), "hipEventRecord");
        HIP_TRY(hipStreamWaitEvent(b->aux, b->fork, 0), "hipStreamWaitEvent");
        Launch S = L;
        S.op = OP_STEP_BATCH_SLOW;
        S.grid = grid_for(b->n_slow, 256);
        S.block = 256;
        S.wave_cav = b->d_wave_cav;
        S.slow_list = b->d_slow;
        S.n_slow = b->n_slow;
        hipError_t e = b->launch(S, b->aux);
        if (e != hipSuccess) return hip_fail(e, "batch edge-cell launch");
        HIP_TRY(hipEventRecord(b->join, b->aux), "hipEventRecord");
    }
    if (L.grid > 0) {
        hipError_t e = b->launch(L, b->stream);
        if (e != hipSuccess) return hip_fail(e, "batch step launch");
    }
    if (edge) HIP_TRY(hipStreamWaitEvent(b->stream, b->join, 0), "hipStreamWaitEvent");
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
        hipError_t e = b->launch(L, b->stream);
        if (e != hipSuccess) return hip_fail(e, "batch init launch");
    }
    b->phase = 0;
    b->cur = 0;
    return LBM_OK;
}

// Field of cavity idx holding the current state, and whether a read-out must
// apply the pending gather first (AA after an odd count, pull after a step).
Field current_field(const lbm_batch* b, int idx, int* pending)
{
    *pending = (b->scheme == LBM_AA || b->scheme == LBM_2POP_PULL) ? b->phase : 0;
    Field F = b->cav[b->scheme == LBM_AA ? 0 : b->cur][idx].F;
    F.out = nullptr;
    return F;
}

float time_steps(lbm_batch* b, int warm, int timed, hipEvent_t e0, hipEvent_t e1, int* rc)
{
    for (int s = 0; s < warm && !*rc; ++s) *rc = launch_batch_step(b);
    if (*rc) return 0.f;
    if (hipEventRecord(e0, b->stream) != hipSuccess) return *rc = fail(LBM_EDEVICE, "hipEventRecord"), 0.f;
    for (int s = 0; s < timed && !*rc; ++s) *rc = launch_batch_step(b);
    if (*rc) return 0.f;
    float ms = 0.f;
    if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        return *rc = fail(LBM_EDEVICE, "batch autotune timing"), 0.f;
    return ms;
}

// Autotuner of the fast kernel's launch shape: block size and cells per
// thread first (at the storage type's residency cap, tiles split by XCD),
// then the residency cap at the best of those, then the split on or off.
// Each candidate is timed over an even number of steps, so AA and 2Pop
// kinds alternate as they do in a run.
int autotune_batch(lbm_batch* b)
{
    static const int blocks[] = {128, 256, 512, 1024};
    static const int cpts[] = {1, 2, 4};
    static const int caps[] = {-1, 0, 2, 3, 4, 6};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
    int rc = LBM_OK;
    float best = 1e30f;
    int bb = 256, bc = 1, bw = -1;
    const int maxb = max_step_block(19, b->collision, b->elem);
    b->waves = -1;
    b->xcd = 1;
    for (int blk : blocks) {
        if (blk > maxb) continue;
        for (int c : cpts) {
            rc = build_tiles(b, blk, c);
            if (rc) break;
            const float ms = time_steps(b, 2, 6, e0, e1, &rc);
            if (rc) break;
            if (ms < best) best = ms, bb = blk, bc = c;
        }
        if (rc) break;
    }
    if (!rc) rc = build_tiles(b, bb, bc);
    for (int w : caps) {
        if (rc || w == -1) continue;
        b->waves = w;
        const float ms = time_steps(b, 2, 6, e0, e1, &rc);
        if (!rc && ms < best) best = ms, bw = w;
    }
    b->waves = bw;
    if (!rc) {
        b->xcd = 0;
        const float ms = time_steps(b, 2, 6, e0, e1, &rc);
        if (rc || !(ms < best)) b->xcd = 1;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
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

// Cache line "key block cells_per_thread waves xcd"; the last match wins.
bool cached_shape(const char* path, const std::string& key, int* block, int* cpt, int* waves, int* xcd)
{
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512], k[256];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        int blk = 0, c = 0, w = 0, x = 0;
        if (std::sscanf(line, "%255s %d %d %d %d", k, &blk, &c, &w, &x) != 5 || key != k) continue;
        if (blk >= 64 && blk <= 1024 && blk % 64 == 0 && (c == 1 || c == 2 || c == 4) && w >= -1 && w <= 8 &&
            (x == 0 || x == 1)) {
            *block = blk, *cpt = c, *waves = w, *xcd = x;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void free_batch(lbm_batch* b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->aux) (void)hipStreamSynchronize(b->aux);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->d_cav[0]) (void)hipFree(b->d_cav[0]);
    if (b->d_cav[1]) (void)hipFree(b->d_cav[1]);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_slow) (void)hipFree(b->d_slow);
    if (b->d_wave_cav) (void)hipFree(b->d_wave_cav);
    if (b->pool) (void)hipFree(b->pool);
    if (b->flags) (void)hipFree(b->flags);
    if (b->partial) (void)hipFree(b->partial);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
    if (b->aux) (void)hipStreamDestroy(b->aux);
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
    if (scheme != LBM_2POP && scheme != LBM_AA && scheme != LBM_2POP_PULL) {
        fail(scheme == LBM_SWAP ? LBM_EUNSUPPORTED : LBM_EINVAL, "batch schemes: 2Pop, AA or 2Pop pull");
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
    lbm_batch_opts o{};
    if (opts) o = *opts;
    if (o.block_size && (o.block_size % 64 || o.block_size < 64 || o.block_size > 1024)) {
        fail(LBM_EINVAL, "block_size must be a multiple of 64 up to 1024");
        return nullptr;
    }
    if (o.cells_per_thread && o.cells_per_thread != 1 && o.cells_per_thread != 2 && o.cells_per_thread != 4) {
        fail(LBM_EINVAL, "cells_per_thread must be 0, 1, 2 or 4");
        return nullptr;
    }
    if (o.waves_per_simd < -1 || o.waves_per_simd > 8) {
        fail(LBM_EINVAL, "waves_per_simd must lie in [-1, 8]");
        return nullptr;
    }
    if (o.xcd_split < 0 || o.xcd_split > 2) {
        fail(LBM_EINVAL, "xcd_split must be 0 (on), 1 (on) or 2 (off)");
        return nullptr;
    }
    lbm_batch* b = new lbm_batch();
    b->count = count;
    b->scheme = scheme;
    b->collision = collision;
    b->elem = storage_dtype == LBM_F64 ? 8 : storage_dtype == LBM_F32_SHIFTED ? 4 : 2;
    b->no_residency_cap = std::getenv("LBM_NO_RESIDENCY_CAP") != nullptr;
    b->dtype = storage_dtype;
    b->desc.assign(d, d + count);
    b->opts = o;
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
    {
        hipError_t e = hipStreamCreateWithFlags(&b->aux, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming);
        if (e != hipSuccess) {
            hip_fail(e, "batch stream and events");
            return bail(0);
        }
    }

    // Pool layout: per cavity Q*stride elements (x2 for 2Pop and pull), 256-byte aligned.
    const bool two = scheme == LBM_2POP || scheme == LBM_2POP_PULL;
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
        total += bytes * (two ? 2 : 1);
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
        const double lid[3] = {d[c].u_lid, 0.0, 0.0};
        F.lid = lid_terms(Q, (int)s, lid);
        RelaxD r{};
        r.omega = d[c].omega;
        const double lam = d[c].trt_lambda > 0.0 ? d[c].trt_lambda : 0.25;
        r.omega_m = collision == LBM_TRT ? 1.0 / (0.5 + lam / (1.0 / d[c].omega - 0.5)) : d[c].omega;
        r.omega_b = d[c].omega;
        r.omega3 = 1.0;
        r.omega4 = 1.0;
        b->cav[0][c] = BatchCavity{F, r};
    }
    b->box = scheme != LBM_2POP;
    for (int c = 0; c < count; ++c) b->box = b->box && b->cav[0][c].F.ntot < (1u << 24);
    b->order.resize(count);
    for (int c = 0; c < count; ++c) b->order[c] = c;
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](int x, int y) { return b->cav[0][x].F.ntot > b->cav[0][y].F.ntot; });
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
        B.F.out = two ? (char*)b->pool + off[c] + bytes + skip : nullptr;
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
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        hip_fail(e, "batch tables");
        return bail(0);
    }
    if (build_slow_list(b, ftotal) || init_batch_state(b)) return bail(0);
    const int maxb = max_step_block(19, b->collision, b->elem);
    const int block = std::min(b->opts.block_size > 0 ? b->opts.block_size : 256, maxb);
    b->waves = b->opts.waves_per_simd;
    b->xcd = b->opts.xcd_split == 2 ? 0 : 1;
    if (build_tiles(b, block, b->opts.cells_per_thread > 0 ? b->opts.cells_per_thread : 1)) return bail(0);
    if (b->opts.autotune) {
        const std::string key = b->opts.autotune_cache ? cache_key(b) : std::string();
        int hb = 0, hc = 1, hw = -1, hx = 1;
        if (b->opts.autotune_cache && cached_shape(b->opts.autotune_cache, key, &hb, &hc, &hw, &hx) && hb <= maxb) {
            b->waves = hw;
            b->xcd = hx;
            if (build_tiles(b, hb, hc)) return bail(0);
        } else {
            if (autotune_batch(b) || init_batch_state(b)) return bail(0);
            if (b->opts.autotune_cache) {
                if (FILE* f = std::fopen(b->opts.autotune_cache, "a")) {
                    std::fprintf(f, "%s %d %d %d %d\n", key.c_str(), b->block, b->cpt, b->waves, b->xcd);
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
    const int phase0 = b->phase, cur0 = b->cur;
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    int rc = LBM_OK;
    for (int s = 0; s < b->opts.graph_steps && !rc; ++s) rc = launch_batch_step(b);
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    b->phase = phase0;  // capture only recorded the launches
    b->cur = cur0;
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    b->graph_steps = b->opts.graph_steps;
    b->graph_phase = phase0;
    b->graph_cur = cur0;
    return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int n)
{
    if (!b) return fail(LBM_EINVAL, "null batch");
    if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
    if (b->opts.use_graph) {
        // 2Pop pull: the entry step (AA even) runs eagerly, so that a graph
        // holds pull steps only and its even count returns the arrays.
        if (b->scheme == LBM_2POP_PULL && !b->phase && n >= b->opts.graph_steps) {
            int rc = launch_batch_step(b);
            if (rc) return rc;
            --n;
        }
        while (n >= b->opts.graph_steps) {
            if (!b->graph || b->graph_phase != b->phase || b->graph_cur != b->cur) {
                int rc = capture_graph(b);
                if (rc) return rc;
            }
            HIP_TRY(hipGraphLaunch(b->graph, b->stream), "hipGraphLaunch");
            n -= b->graph_steps;  // graph_steps is even: phase and array are unchanged
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
        const int cur = b->cur;  // the array the step reads
        const BatchCavity* table = nullptr;
        const int kind = next_step(b, &table);
        for (int c = 0; c < b->count; ++c) {
            Launch L{};
            L.op = OP_STEP_ALL;
            L.model = b->collision;
            L.layout = LAYOUT_SOA;
            L.block = 256;
            L.grid = grid_for(b->cav[0][c].F.ntot, 256);
            L.F = b->cav[b->scheme == LBM_AA ? 0 : cur][c].F;
            L.relax = b->cav[0][c].relax;
            L.kind = kind;
            hipError_t e = b->launch(L, b->stream);
            if (e != hipSuccess) return hip_fail(e, "sequential step launch");
        }
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

int lbm_batch_launch_shape(lbm_batch* b, int* block_size, int* cells_per_thread, int* waves_per_simd,
                           int* xcd_split, int64_t* edge_cells)
{
    if (!b) return fail(LBM_EINVAL, "null batch");
    if (xcd_split) *xcd_split = b->xcd;
    if (block_size) *block_size = b->block;
    if (cells_per_thread) *cells_per_thread = b->cpt;
    if (waves_per_simd) *waves_per_simd = b->waves;
    if (edge_cells) *edge_cells = b->n_edge;
    return LBM_OK;
}

int lbm_batch_sync(lbm_batch* b)
{
    if (!b) return fail(LBM_EINVAL, "null batch");
    HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    return LBM_OK;
}

}  // extern "C"
