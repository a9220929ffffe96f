// Host runtime and C ABI of the lattice Boltzmann library (include/lbm.h).
//
// A handle owns (or borrows) the population array(s) and the flag array,
// keeps the AA phase and step counter, and enqueues kernels on its stream.
// Every launch goes through the (Q, storage) translation unit that holds the
// kernel instantiations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"
#include "lattice.hpp"
#include "lbm.h"

using namespace lbm;

namespace {
thread_local std::string g_error;
}

namespace lbm_detail {
int set_error(int code, const std::string& msg)
{
    g_error = msg;
    return code;
}
}  // namespace lbm_detail

namespace {

int fail(int code, const std::string& msg)
{
    g_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

using LaunchFn = hipError_t (*)(const Launch&, hipStream_t);

LaunchFn pick_tu(int q, int dtype)
{
    if (q == 19) return dtype == LBM_F64 ? launch_q19_f64 : dtype == LBM_F32_SHIFTED ? launch_q19_f32 : launch_q19_f16;
    return dtype == LBM_F64 ? launch_q27_f64 : dtype == LBM_F32_SHIFTED ? launch_q27_f32 : launch_q27_f16;
}

size_t elem_bytes(int dtype) { return dtype == LBM_F64 ? 8 : dtype == LBM_F32_SHIFTED ? 4 : 2; }

// SoA stride: the cell count rounded up to 1024 elements, so that every
// population stream starts on a fresh 2-8 KiB boundary, plus a padding picked
// at creation. How the 19/27 stream bases fall on the HBM channels depends on
// the stride in a way no simple rule captures (measured, FP64 AA: a 320^3
// cavity runs at 14.0 k MLUPS unpadded and 16.8 k with 1024 elements of
// padding, while 256^3 is best unpadded), so large lattices time a few
// candidates. Buffers always reserve room for the largest.
static constexpr int64_t kStridePads[] = {0, 256, 1024, 3072};
static constexpr int64_t kMaxStridePad = 3072;

int64_t soa_stride(int64_t ntot)
{
    const int64_t a = 1024;
    int64_t s = (ntot + a - 1) / a * a;
    if (const char* e = std::getenv("LBM_STRIDE_PAD")) s += std::max<int64_t>(0, std::min<int64_t>(std::atoll(e), kMaxStridePad));
    return s;
}

// SoA halo: padding (elements) before the first and after the last stream,
// at least the largest neighbour offset ny*nz + nz + 1, so that a shifted
// access i +- d_k of any cell stays inside the allocation.
int64_t soa_halo(int ny, int nz)
{
    const int64_t h = (int64_t)ny * nz + nz + 1;
    return (h + 255) / 256 * 256;
}

}  // namespace

// The lid terms w_k = -6 t_k c_k . u (Eq. storage2, rho_w = 1) of the
// built-in geometries, rounded to the storage type the way an FP32 value is
// stored: FP64 as is, FP32 once, FP16 through FP32.
LidTerms lbm::lid_terms(int q, int elem_bytes, const double u[3])
{
    LidTerms t{};
    int32_t c[27][3];
    double w[27];
    int32_t opp[27];
    lbm_lattice(q, &c[0][0], w, opp);
    for (int k = 0; k < q; ++k) {
        const double cu = c[k][0] * u[0] + c[k][1] * u[1] + c[k][2] * u[2];
        const double v = -6.0 * w[k] * cu;
        t.d[k] = v;
        t.f[k] = elem_bytes == 2 ? (float)(_Float16)(float)v : (float)v;
    }
    return t;
}

namespace {

// Blocked layout: padding cells before cell 0 (whole blocks covering the
// largest neighbour offset) and the values of the whole array.
int64_t blocked_pad(int ny, int nz)
{
    const int64_t h = (int64_t)ny * nz + nz + 1;
    return (h + kBlockCells - 1) / kBlockCells * kBlockCells;
}
uint64_t blocked_values(int64_t ntot, int ny, int nz, int q)
{
    const uint64_t cells = (uint64_t)((ntot + kBlockCells - 1) / kBlockCells * kBlockCells + 2 * blocked_pad(ny, nz));
    return cells * (uint64_t)q;
}

double trt_omega_minus(double omega, double lambda)
{
    return 1.0 / (0.5 + lambda / (1.0 / omega - 0.5));
}

// --- flag construction ------------------------------------------------------

__global__ void k_flag_types(uint8_t* fl, int nx, int ny, int nz, int geometry)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t n = (uint64_t)nx * ny * nz;
    if (i >= n) return;
    const int z = (int)(i % nz), y = (int)((i / nz) % ny), x = (int)(i / ((uint64_t)ny * nz));
    uint8_t t = FL_FLUID;
    if (geometry == LBM_CAVITY) {
        const bool inside = x >= 1 && x <= nx - 2 && y >= 1 && y <= ny - 2 && z >= 1 && z <= nz - 2;
        if (!inside) t = z == nz - 1 ? FL_LID : FL_WALL;
    } else if (geometry == LBM_CHANNEL) {
        if (z == 0) t = FL_WALL;
        else if (z == nz - 1) t = FL_LID;
    }
    fl[i] = t;
}

// Fast-path hints of a fluid cell, from its 26 neighbours (wrapping):
// BORDER on a box face; a wall-plane code when the non-fluid neighbours are
// exactly the nine on one side and none is a pressure wall (the fast kernels
// bounce those back themselves; `no_planes`: never, as with curved walls);
// NEARWALL for any other pattern of non-fluid neighbours.
__global__ void k_flag_hints(uint8_t* fl, int nx, int ny, int nz, int no_planes)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t n = (uint64_t)nx * ny * nz;
    if (i >= n) return;
    if ((fl[i] & FL_TYPE) != FL_FLUID) return;
    const int z = (int)(i % nz), y = (int)((i / nz) % ny), x = (int)(i / ((uint64_t)ny * nz));
    const bool border = x == 0 || x == nx - 1 || y == 0 || y == ny - 1 || z == 0 || z == nz - 1;
    int total = 0, pressure = 0, side[3][2] = {{0, 0}, {0, 0}, {0, 0}};  // solid neighbours at d_axis = -1 / +1
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                const int xx = (x + dx + nx) % nx, yy = (y + dy + ny) % ny, zz = (z + dz + nz) % nz;
                const uint64_t j = ((uint64_t)xx * ny + yy) * nz + zz;
                if ((fl[j] & FL_TYPE) == FL_FLUID) continue;
                ++total;
                pressure += (fl[j] & FL_TYPE) == FL_PRESSURE;
                const int d[3] = {dx, dy, dz};
                for (int a = 0; a < 3; ++a)
                    if (d[a]) ++side[a][d[a] > 0];
            }
    uint8_t h = 0;
    if (border) {
        h = FL_BORDER | (total ? FL_NEARWALL : 0);
        if (!total && nz >= 3 && (z == 0 || z == nz - 1) && x > 0 && x < nx - 1 && y > 0 && y < ny - 1) h |= FL_ZWRAP;
    } else if (total) {
        h = FL_NEARWALL;
        for (int a = 0; a < 3 && !pressure && !no_planes; ++a)
            for (int sgn = 0; sgn < 2; ++sgn)
                if (total == 9 && side[a][sgn] == 9) h = (uint8_t)((1 + 2 * a + sgn) << FL_PLANE_SHIFT);
    }
    fl[i] |= h;
}

__global__ void k_flag_types_only(const uint8_t* fl, uint8_t* out, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = fl[i] & FL_TYPE;
}

// Caller cell types: count the cells that break the rules (type not FLUID /
// WALL / LID / PRESSURE; a fluid cell on a box face whose axis does not wrap; a wall
// velocity of magnitude >= 0.4 or a wall density outside (0, 10)).
__global__ void k_check_geometry(const uint8_t* type, const double* wu, const double* wr, int nx, int ny, int nz,
                                 int wrap_x, int wrap_y, int wrap_z, unsigned long long* bad)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t n = (uint64_t)nx * ny * nz;
    bool err = false;
    if (i < n) {
        const int z = (int)(i % nz), y = (int)((i / nz) % ny), x = (int)(i / ((uint64_t)ny * nz));
        const uint8_t t = type[i];
        if (t > FL_PRESSURE) err = true;
        if (t == FL_FLUID) {
            if (!wrap_x && (x == 0 || x == nx - 1)) err = true;
            if (!wrap_y && (y == 0 || y == ny - 1)) err = true;
            if (!wrap_z && (z == 0 || z == nz - 1)) err = true;
        } else {
            if (wu) {
                const double a = wu[i], b = wu[n + i], c = wu[2 * n + i];
                if (!(a * a + b * b + c * c < 0.16)) err = true;
            }
            if (wr && !(wr[i] > 0.0 && wr[i] < 10.0)) err = true;
        }
    }
    const unsigned long long m = __ballot(err);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(bad, (unsigned long long)__popcll(m));
}

// Curved-wall distances: count values outside (0, 1] and values other than
// 1/2 (two counters).
__global__ void k_check_qlink(const double* q, uint64_t n, unsigned long long* cnt)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool bad = i < n && !(q[i] > 0.0 && q[i] <= 1.0);
    const bool curved = i < n && q[i] != 0.5;
    const unsigned long long mb = __ballot(bad), mc = __ballot(curved);
    if ((threadIdx.x & 63) == 0) {
        if (mb) atomicAdd(&cnt[0], (unsigned long long)__popcll(mb));
        if (mc) atomicAdd(&cnt[1], (unsigned long long)__popcll(mc));
    }
}

__global__ void k_clear_hints(uint8_t* fl, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) fl[i] &= FL_TYPE;
}

__global__ void k_set_types(const uint8_t* type, uint8_t* fl, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) fl[i] = type[i];
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }

__global__ void k_count_fluid(const uint8_t* fl, uint64_t n, unsigned long long* count)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool f = i < n && (fl[i] & FL_TYPE) == FL_FLUID;
    const unsigned long long b = __ballot(f);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, (unsigned long long)__popcll(b));
}

// Sum per-block partial pairs in a fixed order (one block of 256 threads).
__global__ void __launch_bounds__(256) k_reduce_pairs(const double* partial, int nblocks, double* result)
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

uint32_t grid_for(uint64_t n, int block) { return (uint32_t)((n + block - 1) / block); }

// Streaming copy: one 16-byte vector per lane, one thread per vector, stores
// nontemporal (the configuration that measured fastest on gfx950); a
// grid-stride loop only beyond 2^31 vectors.
__global__ void __launch_bounds__(256) k_copy16(uint4* __restrict__ dst, const uint4* __restrict__ src, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint4 v = src[i];
        __builtin_nontemporal_store(v.x, &dst[i].x);
        __builtin_nontemporal_store(v.y, &dst[i].y);
        __builtin_nontemporal_store(v.z, &dst[i].z);
        __builtin_nontemporal_store(v.w, &dst[i].w);
    }
}

// Copy of NS separate FP64 streams, one element of each per lane: the memory
// pattern of the local step kernels (all loads of a cell issued, then all its
// stores) without their arithmetic or flags. With shifts, stream s is read at
// i - d_s and written at i + d_s, d_s the offset of the lattice velocity c_s
// (the AA odd step's pattern).
template <int NS>
__global__ void __launch_bounds__(256) k_copy_streams(double* __restrict__ dst, const double* __restrict__ src,
                                                      uint64_t stride, uint32_t n, int ny, int nz)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v[NS];
    const bool shifted = nz > 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int64_t d = shifted ? ((int64_t)L<NS>::cx(s) * ny + L<NS>::cy(s)) * nz + L<NS>::cz(s) : 0;
        v[s] = src[(int64_t)(s * stride + i) - d];
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) asm volatile("" : "+v"(v[s]));
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int64_t d = shifted ? ((int64_t)L<NS>::cx(s) * ny + L<NS>::cy(s)) * nz + L<NS>::cz(s) : 0;
        dst[(int64_t)(s * stride + i) + d] = v[s];
    }
}

// Memory-pattern probe over the D3Q19 streams, FP64: value (s, j) at
// s * stride + j (SoA, LB = 0) or in blocks of 2^LB cells holding all 19
// streams, ((j >> LB) * 19 + s) << LB | (j & (2^LB - 1)). PAT 0: read and
// write cell i (the local kinds); 1: read i - d_s, write i (2Pop pull);
// 2: read i - d_s, write i + d_s (AA odd). VEC consecutive cells per lane
// (SoA). All loads of a lane are issued before its stores, as in the step
// kernels; nothing else is done with the values.
template <int LB>
__device__ __forceinline__ int64_t probe_at(int64_t j, int s, uint64_t stride)
{
    if constexpr (LB == 0) return (int64_t)s * (int64_t)stride + j;
    else return ((j >> LB) * 19 + s) * ((int64_t)1 << LB) + (j & ((1 << LB) - 1));
}

template <int LB, int PAT, int VEC>
__global__ void __launch_bounds__(256) k_pattern_copy(double* __restrict__ dst, const double* __restrict__ src,
                                                      uint64_t stride, uint32_t n, int ny, int nz)
{
    typedef double V __attribute__((ext_vector_type(VEC), aligned(8)));
    const uint32_t i = (blockIdx.x * blockDim.x + threadIdx.x) * VEC;
    if (i + VEC > n) return;
    V v[19];
#pragma unroll
    for (int s = 0; s < 19; ++s) {
        const int64_t d = PAT ? ((int64_t)L<19>::cx(s) * ny + L<19>::cy(s)) * nz + L<19>::cz(s) : 0;
        v[s] = *reinterpret_cast<const V*>(src + probe_at<LB>((int64_t)i - d, s, stride));
    }
#pragma unroll
    for (int s = 0; s < 19; ++s)
#pragma unroll
        for (int c = 0; c < VEC; ++c) {
            double t = v[s][c];
            asm volatile("" : "+v"(t));
            v[s][c] = t;
        }
#pragma unroll
    for (int s = 0; s < 19; ++s) {
        const int64_t d = PAT == 2 ? ((int64_t)L<19>::cx(s) * ny + L<19>::cy(s)) * nz + L<19>::cz(s) : 0;
        *reinterpret_cast<V*>(dst + probe_at<LB>((int64_t)i + d, s, stride)) = v[s];
    }
}

template <int LB, int PAT>
void launch_pattern(int vec, uint32_t grid, uint32_t lds, hipStream_t st, double* dst, const double* src,
                    uint64_t stride, uint32_t n, int ny, int nz)
{
    if (vec == 2) k_pattern_copy<LB, PAT, 2><<<grid, 256, lds, st>>>(dst, src, stride, n, ny, nz);
    else k_pattern_copy<LB, PAT, 1><<<grid, 256, lds, st>>>(dst, src, stride, n, ny, nz);
}

}  // namespace

// --- scratch of the no-allocation invariants entry point -----------------------
// lbm_invariants_noalloc keeps its per-block partial sums (two per block of
// 256 cells) and, for host outputs, its two results in this file-scope device
// array instead of the handle's reduction buffer, so that the call allocates
// nothing. It serves lattices of up to kNoAllocMaxCells cells. Each GPU holds
// its own copy, at its own address, until the process ends. In host code the
// name `scratch` is only a stand-in: its device address is looked up once per
// device at handle creation (hipGetSymbolAddress, that device current), and
// only that address is ever passed to kernels or copies.
constexpr int64_t kNoAllocMaxCells = int64_t(1) << 25;
constexpr size_t kNoAllocDoubles = 2 * (size_t)(kNoAllocMaxCells / 256) + 2;
constexpr int kNoAllocMaxDevices = 64;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[kNoAllocMaxDevices] = {};  // device address of `scratch`, per device

// Device address of `scratch` on the current device (looked up on first use).
int scratch_address(int device, double** out)
{
    if (device < 0 || device >= kNoAllocMaxDevices)
        return fail(LBM_EUNSUPPORTED, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[device] = (double*)p;
    }
    *out = g_scratch_ptr[device];
    return LBM_OK;
}
}  // namespace

// --- handle --------------------------------------------------------------------

// ceil(2^64 / d) for d >= 2, else 0. The high word of i * ceil(2^64 / d) is
// floor(i / d) for every 32-bit i: it exceeds i / d by less than i / 2^64 <
// 2^-32 <= 1/d, too little to carry past the next integer.
static uint64_t reciprocal64(int d) { return d >= 2 ? ~0ull / (uint64_t)d + 1 : 0; }

// Schemes with a second population array.
static bool two_arrays(int scheme) { return scheme == LBM_2POP || scheme == LBM_2POP_PULL; }

struct lbm_handle {
    lbm_desc d;
    int q = 19;
    int64_t ntot = 0, fluid = 0, stride = 0;
    size_t pop_bytes = 0, out_bytes = 0, flag_bytes = 0;
    void* pop_alloc = nullptr;  // allocations (or caller buffers) as given
    void* out_alloc = nullptr;
    void* pop = nullptr;        // cell 0 of stream 0 (past the SoA halo)
    void* out = nullptr;
    uint8_t* flags = nullptr;
    bool own_pop = false, own_out = false, own_flags = false;
    hipStream_t stream = nullptr;
    RelaxD relax{};
    int aa_phase = 0;
    int64_t steps = 0;
    int64_t first_nonfinite = -1;
    int block = 256;
    double* partial = nullptr;  // invariant partial sums (2 per block) + 2 results
    int red_blocks = 0;
    int device = 0;                 // GPU the buffers live on (current at creation)
    double* scratch = nullptr;      // that GPU's copy of `scratch` (lbm_invariants_noalloc)
    uint32_t* slow_list = nullptr;  // fluid cells off the fast path, ascending
    uint32_t n_slow = 0;
    uint32_t* slow_list_z = nullptr;  // the same without the z-wrap cells, which the fast
    uint32_t n_slow_z = 0;            // pull and AA odd kernels handle (one allocation)
    int cpt = 1;                    // cells per lane of the fast step kernels
    hipStream_t aux = nullptr;      // runs the near-wall part beside the fast part
    hipEvent_t fork = nullptr, join = nullptr;
    LaunchFn launch = nullptr;
    bool lds_override = false;      // LBM_STEP_LDS given: fixed dynamic LDS of the fast
    uint32_t lds_local = 0;         //   kernels of local kinds
    uint32_t lds_neighbour = 0;     //   and of the kinds that reach neighbours
    bool custom_walls = false;      // wall terms set per cell (lbm_set_geometry)
    int pull_kernel = 0;            // LBM_PULL_KERNEL: 0 by measurement, 1 flag-driven ("flag"),
                                    //   2 position-driven on the built-in cavity ("box")
    int aa_kernel = 0;              // LBM_AA_KERNEL, the same for the AA odd kind
    double* qlink = nullptr;        // curved-wall distances q[k][ntot] (lbm_set_wall_distances)
    bool reverse_blocks = false;    // LBM_REVERSE_BLOCKS: step kernels visit cells in reverse order
    bool use_graph = false;         // small lattice: replay captured steps
    bool fused = false;             // one kernel per kind (fast and edge parts together)
    hipStream_t cap = nullptr;      // private stream the step graph is captured on
    hipGraphExec_t graph = nullptr;
    int graph_phase = -1;           // AA phase and 2Pop buffer the graph starts from
    void* graph_pop = nullptr;

    // SoA whose streams, with a neighbour offset's reach on either side, span
    // under 4 GiB: the position-driven kernels then address it by 32-bit byte
    // offsets from one base.
    bool soa32() const
    {
        const uint64_t h = (uint64_t)d.ny * d.nz + d.nz + 1;
        return d.layout == LBM_SOA &&
               ((uint64_t)q * (uint64_t)stride + 2 * h) * elem_bytes(d.storage_dtype) < (1ull << 32);
    }
    Field field() const
    {
        Field F;
        F.pop = pop;
        F.out = out;
        F.flags = flags;
        F.stride = stride;
        F.ntot = (uint32_t)ntot;
        F.nx = d.nx;
        F.ny = d.ny;
        F.nz = d.nz;
        F.reverse = reverse_blocks ? 1 : 0;
        F.custom_walls = custom_walls ? 1 : 0;
        F.qlink = qlink;
        F.lid = lid_terms(q, (int)elem_bytes(d.storage_dtype), d.lid_velocity);
        F.zrecip = reciprocal64(d.nz);
        F.yrecip = reciprocal64(d.ny);
        F.soa32 = soa32() ? 1 : 0;
        F.run_rows = d.layout == LBM_BLOCKED && d.nz == (int)kBlockCells ? 1 : 0;
        return F;
    }
    Launch base(int op) const
    {
        Launch L{};
        L.op = op;
        L.model = d.collision;
        L.layout = d.layout;
        L.block = block;
        L.grid = grid_for((uint64_t)ntot, block);
        L.F = field();
        L.relax = relax;
        return L;
    }
};

// Whether the stored state is post-collision in slot kbar (AA after an even
// step, 2Pop pull after any step): read-outs then apply the pending gather.
static int pending_gather(const lbm_handle* h)
{
    return (h->d.scheme == LBM_AA || h->d.scheme == LBM_2POP_PULL) ? h->aa_phase : 0;
}

extern "C" {

const char* lbm_last_error(void) { return g_error.c_str(); }

void lbm_desc_default(lbm_desc* d)
{
    std::memset(d, 0, sizeof(*d));
    d->lattice = 19;
    d->nx = d->ny = d->nz = 8;
    d->scheme = LBM_AA;
    d->collision = LBM_BGK;
    d->storage_dtype = LBM_F64;
    d->layout = LBM_SOA;
    d->geometry = LBM_CAVITY;
    d->ptr_kind = LBM_PTR_DEVICE;
    d->omega = 1.0;
    d->trt_lambda = 0.25;
    d->omega_bulk = 0.0;
}

static int validate(const lbm_desc* d)
{
    if (!d) return fail(LBM_EINVAL, "null description");
    if (d->lattice != 19 && d->lattice != 27) return fail(LBM_EINVAL, "lattice must be 19 or 27");
    const int lo = d->geometry == LBM_CAVITY ? 3 : 1;
    if (d->nx < lo || d->ny < lo || d->nz < lo)
        return fail(LBM_EINVAL, d->geometry == LBM_CAVITY ? "cavity dimensions must be >= 3" : "dimensions must be >= 1");
    if (d->geometry == LBM_CHANNEL && d->nz < 3) return fail(LBM_EINVAL, "channel needs nz >= 3");
    const int64_t n = (int64_t)d->nx * d->ny * d->nz;
    if (n > 0x7fffffffLL) return fail(LBM_EUNSUPPORTED, "more than 2^31-1 cells");
    if (d->layout == LBM_SOA && (uint64_t)n * elem_bytes(d->storage_dtype) >= (1ull << 32))
        return fail(LBM_EUNSUPPORTED, "SoA streams above 4 GiB (cells x bytes per value) are not supported");
    if (d->scheme < LBM_2POP || d->scheme > LBM_2POP_PULL) return fail(LBM_EINVAL, "unknown scheme");
    if (d->collision < LBM_BGK || d->collision > LBM_K) return fail(LBM_EINVAL, "unknown collision model");
    if (d->collision == LBM_K && d->lattice != 19)
        return fail(LBM_EUNSUPPORTED, "the cumulant model is defined on D3Q19 only");
    if (d->storage_dtype < LBM_F64 || d->storage_dtype > LBM_F16_SHIFTED) return fail(LBM_EINVAL, "unknown storage dtype");
    if (d->layout != LBM_SOA && d->layout != LBM_AOS && d->layout != LBM_BLOCKED) return fail(LBM_EINVAL, "unknown layout");
    if (d->layout == LBM_BLOCKED && blocked_values(n, d->ny, d->nz, d->lattice) * elem_bytes(d->storage_dtype) >= (1ull << 32))
        return fail(LBM_EUNSUPPORTED, "blocked layout above 4 GiB per population array is not supported");
    if (d->geometry < LBM_CAVITY || d->geometry > LBM_CHANNEL) return fail(LBM_EINVAL, "unknown geometry");
    if (d->ptr_kind != LBM_PTR_DEVICE && d->ptr_kind != LBM_PTR_HOST) return fail(LBM_EINVAL, "unknown pointer kind");
    if (!(d->omega > 0.0 && d->omega < 2.0)) return fail(LBM_EINVAL, "omega must lie in (0, 2)");
    if (d->omega_bulk > 0.0 && !(d->omega_bulk < 2.0)) return fail(LBM_EINVAL, "omega_bulk must lie in (0, 2)");
    if (d->omega3 > 0.0 && !(d->omega3 < 2.0)) return fail(LBM_EINVAL, "omega3 must lie in (0, 2)");
    if (d->omega4 > 0.0 && !(d->omega4 < 2.0)) return fail(LBM_EINVAL, "omega4 must lie in (0, 2)");
    if (d->collision == LBM_TRT && !(d->trt_lambda > 0.0)) return fail(LBM_EINVAL, "trt_lambda must be > 0");
    const double* v = d->lid_velocity;
    if (!(std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) < 0.4)) return fail(LBM_EINVAL, "|lid velocity| must be < 0.4");
    if (d->block_size != 0 && d->block_size != -1 &&
        (d->block_size < 64 || d->block_size > 1024 || d->block_size % 64 != 0))
        return fail(LBM_EINVAL, "block_size must be a multiple of 64 in [64, 1024] (0 auto, -1 autotune)");
    if (d->check_every < 0) return fail(LBM_EINVAL, "check_every must be >= 0");
    return LBM_OK;
}

int lbm_required_bytes(const lbm_desc* d, size_t out[3])
{
    int rc = validate(d);
    if (rc) return rc;
    if (!out) return fail(LBM_EINVAL, "null output");
    const int64_t n = (int64_t)d->nx * d->ny * d->nz;
    const size_t s = elem_bytes(d->storage_dtype);
    const size_t pop = d->layout == LBM_SOA
                           ? ((size_t)(soa_stride(n) + kMaxStridePad) * d->lattice +
                              2 * (size_t)soa_halo(d->ny, d->nz)) * s
                           : d->layout == LBM_BLOCKED ? (size_t)blocked_values(n, d->ny, d->nz, d->lattice) * s
                                                      : (size_t)n * d->lattice * s;
    out[0] = pop;
    out[1] = two_arrays(d->scheme) ? pop : 0;
    out[2] = (size_t)n;
    return LBM_OK;
}

static int run(lbm_handle* h, const Launch& L)
{
    hipError_t e = h->launch(L, h->stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return LBM_OK;
}

static int init_state(lbm_handle* h, const double* rho, const double* u)
{
    Launch L = h->base(OP_INIT);
    L.init.rho = rho;
    L.init.u = u;
    L.init.keep_walls = h->custom_walls ? 1 : 0;
    int rc = run(h, L);
    if (rc) return rc;
    h->aa_phase = 0;
    h->steps = 0;
    h->first_nonfinite = -1;
    return LBM_OK;
}

// One kernel kind over the lattice: the fast part over all cells, then, for
// the kinds that reach neighbours, the slow part over the listed cells.
static uint32_t step_lds(const lbm_handle* h, int kind, int block)
{
    if (h->lds_override)
        return kind == KIND_AA_ODD || kind == KIND_2POP || kind == KIND_SWAP_STREAM || kind == KIND_PULL ||
                       kind == KIND_PULL_BOX || kind == KIND_AA_ODD_BOX || kind == KIND_PULL_WRAP ||
                       kind == KIND_AA_ODD_WRAP
                   ? h->lds_neighbour : h->lds_local;
    int waves = step_waves((int)elem_bytes(h->d.storage_dtype), kind);
    // The cumulant model's FP64 AA odd step has the most arithmetic per cell
    // and needs the third wave to hide it (15.8 k MLUPS at three, 15.0 k at
    // two, where the other nine models gain 1 % at two).
    if (kind == KIND_AA_ODD_BOX && elem_bytes(h->d.storage_dtype) == 8 && h->d.collision == LBM_K) waves = 3;
    return residency_lds(waves, block);
}

// Kind of the fast launch: the pull and AA odd kinds have variants for
// lattices with z-wrap cells, whose edge list then leaves those cells out.
static bool zwrap_kind(int kind) { return kind == KIND_PULL || kind == KIND_AA_ODD; }

// On the built-in cavity (no caller walls, no curved links) the pull and AA
// odd kinds have position-driven forms with no edge part. The library takes
// them where they measured faster than the flag-driven ones (MLUPS,
// flag-driven -> position-driven):
//   2Pop pull, D3Q19 256^3: FP64 blocked 18.1 k -> 18.9 k (blocks of 128,
//     three per CU, see run_kind); FP32 blocked 34.6 k -> 36.9 k; FP16
//     blocked 67.2 k -> 76.4 k; SoA with 32-bit offsets (arrays under 4 GiB)
//     FP64 16.9 k -> 17.7 k, FP32 34.0 k -> 35.3 k, FP16 61.0 k -> 69.3 k.
//     Not faster: SoA with 64-bit addresses except in FP32 (FP64 16.8 k ->
//     14.0 k, FP16 61.7 k -> 53.8 k, FP32 33.8 k -> 35.6 k).
//   2Pop pull, D3Q27 RR 320^3: blocked FP32 23.5 k -> 25.0 k, FP16 46.7 k ->
//     50.2 k. Slower in SoA (FP32 23.5 k -> 12.0 k, FP16 40.7 k -> 14.7 k).
//   AA, D3Q19 256^3: SoA FP64 16.6 k -> 16.8 k, FP32 33.1 k -> 34.3 k, FP16
//     55.8 k -> 67.0 k; blocked FP64 15.3 k -> 17.1 k, FP32 32.5 k -> 34.3 k,
//     FP16 58.1 k -> 69.1 k.
//   AA, D3Q27 RR 320^3: SoA FP32 20.8 k -> 23.4 k, FP16 32.0 k -> 42.3 k;
//     blocked FP32 20.0 k -> 23.6 k, FP16 34.8 k -> 46.4 k.
// Where the loads are the limit, the work before them (the position, an
// address chosen per lane and direction) can cost more than the second
// round of loads for cells next to a wall, the flag byte and the loads of
// wall lanes that it saves. LBM_PULL_KERNEL and LBM_AA_KERNEL ("box" or
// "flag") override the choice.
static bool box_measured_faster(const lbm_handle* h, int kind)
{
    const size_t s = elem_bytes(h->d.storage_dtype);
    const bool soa = h->d.layout == LBM_SOA, blocked = h->d.layout == LBM_BLOCKED;
    if (kind == KIND_AA_ODD) return (soa || blocked) && (h->q == 19 || s < 8);
    if (kind == KIND_PULL) {
        if (blocked) return s < 8 || h->q == 19;
        return soa && h->q == 19 && (h->soa32() || s == 4);
    }
    return false;
}

// The periodic box (every cell fluid) has position-driven forms of the same
// two kinds, whose wraps come from the cell's position instead of the z-wrap
// flag and the edge-cell list of the x and y faces. Measured on the D3Q19
// 256^3 Taylor-Green box (MLUPS, flag-driven -> position-driven): AA SoA
// FP64 16.9 k -> 17.2 k, FP32 35.0 k -> 34.9 k, FP16 63.3 k -> 67.4 k, AA
// blocked FP16 67.0 k -> 71.1 k; pull blocked FP64 17.4 k -> 17.5 k, FP32
// 35.9 k -> 36.5 k, FP16 73.0 k -> 73.4 k, pull SoA FP16 66.5 k -> 70.1 k.
// D3Q27 keeps the flag-driven kernels (not measured).
static bool wrap_measured_faster(const lbm_handle* h, int kind)
{
    (void)kind;
    return h->q == 19 && (h->d.layout == LBM_SOA || h->d.layout == LBM_BLOCKED);
}

static bool box_kind(const lbm_handle* h, int kind)
{
    if (kind != KIND_PULL && kind != KIND_AA_ODD) return false;
    if (h->custom_walls || h->qlink || h->cpt != 1) return false;
    const int choice = kind == KIND_PULL ? h->pull_kernel : h->aa_kernel;
    if (h->d.geometry == LBM_PERIODIC) return choice == 2 || (choice == 0 && wrap_measured_faster(h, kind));
    return h->d.geometry == LBM_CAVITY && (choice == 2 || (choice == 0 && box_measured_faster(h, kind)));
}

static int fast_kind(const lbm_handle* h, int kind)
{
    if (box_kind(h, kind)) {
        if (h->d.geometry == LBM_PERIODIC) return kind == KIND_PULL ? KIND_PULL_WRAP : KIND_AA_ODD_WRAP;
        return kind == KIND_PULL ? KIND_PULL_BOX : KIND_AA_ODD_BOX;
    }
    if (!zwrap_kind(kind) || h->n_slow_z == h->n_slow) return kind;
    return kind == KIND_PULL ? KIND_PULL_Z : KIND_AA_ODD_Z;
}

static int run_kind(lbm_handle* h, int kind)
{
    Launch L = h->base(OP_STEP);
    L.kind = kind;
    L.lds = step_lds(h, kind, L.block);
    if (h->fused && kind != KIND_SWAP_COLLIDE && kind != KIND_SWAP_STREAM) {
        L.op = OP_STEP_ALL;
        return run(h, L);
    }
    const int cpt = h->cpt;
    const bool neighbours = kind == KIND_2POP || kind == KIND_SWAP_STREAM || kind == KIND_AA_ODD || kind == KIND_PULL;
    const uint32_t n_slow = zwrap_kind(kind) ? h->n_slow_z : h->n_slow;
    if (cpt == 1) {  // one launch, the edge part in the leading blocks
        L.kind = fast_kind(h, kind);
        const size_t s = elem_bytes(h->d.storage_dtype);
        const bool auto_shape = h->d.block_size == 0 && !h->lds_override;
        if (auto_shape && s < 8 && h->q == 19 &&
            ((L.kind == KIND_PULL_BOX && s == 2 && h->d.layout == LBM_BLOCKED) ||
             ((kind == KIND_AA_EVEN || kind == KIND_AA_ODD) && h->d.layout == LBM_SOA && box_kind(h, KIND_AA_ODD)))) {
            // Blocks of 512 at the same resident waves per SIMD, where they
            // measured faster on the 256^3 cavity: FP16 blocked pull 75.3 k ->
            // 77.1 k MLUPS; AA in SoA (both steps) FP32 34.6 k -> 35.2 k, FP16
            // 67.9 k -> 68.6 k. (FP32 pull: 36.8 k -> 36.5 k.)
            L.block = std::min(512, max_step_block(h->q, h->d.collision, (int)s));
            L.grid = grid_for((uint64_t)h->ntot, L.block);
        }
        L.lds = step_lds(h, L.kind, L.block);
        if ((L.kind == KIND_PULL_BOX || L.kind == KIND_PULL_WRAP) && s == 8 && auto_shape) {
            // FP64 position-driven pull: blocks of 128 threads, three per CU
            // (six waves). Measured on the 256^3 cavity, blocked layout:
            // 18.9 k MLUPS, against 18.2 k for blocks of 256 at two waves per
            // SIMD, 18.6 k / 18.4 k for four / five blocks of 128, 17.7 k
            // for six blocks of 64; SoA 17.7 k against 17.4 k; the periodic
            // 256^3 box, blocked: 18.5 k against 17.4 k. (The AA odd kinds
            // measured slower this way.)
            L.block = 128;
            L.grid = grid_for((uint64_t)h->ntot, 128);
            L.lds = residency_lds_blocks(3);
        }
        if (neighbours && n_slow > 0 && L.kind != KIND_PULL_BOX && L.kind != KIND_AA_ODD_BOX &&
            L.kind != KIND_PULL_WRAP && L.kind != KIND_AA_ODD_WRAP) {
            L.slow_list = zwrap_kind(kind) ? h->slow_list_z : h->slow_list;
            L.n_slow = n_slow;
            L.edge_blocks = grid_for(n_slow, L.block);
            L.grid += L.edge_blocks;
        }
        return run(h, L);
    }
    // the vector kernels are compiled for blocks of at most 256
    L.block = std::min(h->block, 256);
    L.grid = grid_for(((uint64_t)h->ntot + cpt - 1) / cpt, L.block);
    L.kind = fast_kind(h, kind);
    int rc = run(h, L);
    if (rc) return rc;
    L.kind = kind;
    // With several cells per lane the fast part skips whole groups, so the
    // listed cells need the second launch for the local kinds as well.
    if ((neighbours || cpt > 1) && n_slow > 0) {
        L.op = OP_STEP_SLOW;
        L.block = 256;
        L.grid = grid_for(n_slow, 256);
        L.slow_list = zwrap_kind(kind) ? h->slow_list_z : h->slow_list;
        L.n_slow = n_slow;
        rc = run(h, L);
    }
    return rc;
}

// The same as two launches, the edge part on a second stream so that its
// scattered, latency-bound accesses overlap the fast part's streaming. Both
// parts touch disjoint memory (every cell owns its locations), and the
// handle's stream waits for the second one before the next launch. Used by
// the kernels with several cells per lane, and on request (LBM_SPLIT_STEP)
// in place of the single launch of run_kind, whose leading blocks overlap the
// parts without the cross-stream wait.
static int run_kind_overlapped(lbm_handle* h, int kind)
{
    const bool neighbours = kind == KIND_2POP || kind == KIND_SWAP_STREAM || kind == KIND_AA_ODD || kind == KIND_PULL;
    const uint32_t n_slow = zwrap_kind(kind) ? h->n_slow_z : h->n_slow;
    if (!h->aux || n_slow == 0 || !(neighbours || h->cpt > 1) || box_kind(h, kind)) return run_kind(h, kind);
    HIP_TRY(hipEventRecord(h->fork, h->stream), "hipEventRecord");
    HIP_TRY(hipStreamWaitEvent(h->aux, h->fork, 0), "hipStreamWaitEvent");
    Launch S = h->base(OP_STEP_SLOW);
    S.kind = kind;
    S.block = 256;
    S.grid = grid_for(n_slow, 256);
    S.slow_list = zwrap_kind(kind) ? h->slow_list_z : h->slow_list;
    S.n_slow = n_slow;
    hipError_t e = h->launch(S, h->aux);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    HIP_TRY(hipEventRecord(h->join, h->aux), "hipEventRecord");
    Launch L = h->base(OP_STEP);
    L.kind = fast_kind(h, kind);
    if (h->cpt > 1) {
        L.block = std::min(h->block, 256);
        L.grid = grid_for(((uint64_t)h->ntot + h->cpt - 1) / h->cpt, L.block);
    }
    L.lds = step_lds(h, kind, L.block);
    int rc = run(h, L);
    if (rc) return rc;
    HIP_TRY(hipStreamWaitEvent(h->stream, h->join, 0), "hipStreamWaitEvent");
    return LBM_OK;
}

static int enqueue_steps(lbm_handle* h, int n)
{
    for (int s = 0; s < n; ++s) {
        int rc;
        if (h->d.scheme == LBM_2POP) {
            rc = run_kind_overlapped(h, KIND_2POP);
            if (rc) return rc;
            std::swap(h->pop, h->out);
        } else if (h->d.scheme == LBM_SWAP) {
            rc = run_kind_overlapped(h, KIND_SWAP_COLLIDE);
            if (!rc) rc = run_kind_overlapped(h, KIND_SWAP_STREAM);
            if (rc) return rc;
        } else if (h->d.scheme == LBM_2POP_PULL && h->aa_phase) {
            // Post-collision state (slot kbar): gather, collide, store into
            // the other array.
            rc = run_kind_overlapped(h, KIND_PULL);
            if (rc) return rc;
            std::swap(h->pop, h->out);
        } else {  // AA; and the first 2Pop-pull step from a pre-collision state
            rc = run_kind_overlapped(h, h->aa_phase ? KIND_AA_ODD : KIND_AA_EVEN);
            if (rc) return rc;
            h->aa_phase ^= 1;
        }
        ++h->steps;
    }
    return LBM_OK;
}

// Small lattices: a step is a few microseconds of GPU work, less than the
// host needs to issue its launches one by one, so the steps are captured once
// in a HIP graph and replayed. A graph holds an even number of steps, so the
// 2Pop buffers and the AA phase come back to where they started. Inside it
// every kernel runs on one stream, and on D3Q19 SoA each kind is a single
// kernel that handles the fast and the edge cells together.
static constexpr int kGraphSteps = 64;
static constexpr int64_t kGraphCells = int64_t(1) << 20;

static int capture_steps(lbm_handle* h)
{
    if (h->graph) {
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
    }
    if (!h->cap) HIP_TRY(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    const int phase0 = h->aa_phase;
    void* const pop0 = h->pop;
    void* const out0 = h->out;
    const int64_t steps0 = h->steps;
    hipStream_t const user = h->stream, aux = h->aux;
    h->stream = h->cap;
    h->aux = nullptr;
    // One launch per step where a fused kernel exists (D3Q19 SoA, one cell per lane).
    h->fused = h->q == 19 && h->d.layout == LBM_SOA && h->cpt == 1;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
    int rc = LBM_OK;
    hipError_t e_end = e;
    if (e == hipSuccess) {
        rc = enqueue_steps(h, kGraphSteps);
        e_end = hipStreamEndCapture(h->cap, &g);
    }
    // The capture only recorded launches: put the host-side state back.
    h->fused = false;
    h->stream = user;
    h->aux = aux;
    h->aa_phase = phase0;
    h->pop = pop0;
    h->out = out0;
    h->steps = steps0;
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    if (rc || e_end != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : hip_fail(e_end, "hipStreamEndCapture");
    }
    e = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    h->graph_phase = phase0;
    h->graph_pop = pop0;
    return LBM_OK;
}

static int enqueue_steps_graph(lbm_handle* h, int n)
{
    // 2Pop pull: the entry step (AA even) goes first, so that a graph holds
    // pull steps only and its even count returns the buffers.
    if (h->d.scheme == LBM_2POP_PULL && !h->aa_phase && n >= kGraphSteps) {
        int rc = enqueue_steps(h, 1);
        if (rc) return rc;
        --n;
    }
    while (n >= kGraphSteps) {
        if (!h->graph || h->graph_phase != h->aa_phase || h->graph_pop != h->pop) {
            int rc = capture_steps(h);
            if (rc) return rc;
        }
        HIP_TRY(hipGraphLaunch(h->graph, h->stream), "hipGraphLaunch");
        h->steps += kGraphSteps;
        n -= kGraphSteps;
    }
    return enqueue_steps(h, n);
}

// Time the candidate stride paddings over a few steps and keep the fastest
// (SoA lattices of at least 2^21 cells; results do not depend on the stride).
static int tune_stride(lbm_handle* h)
{
    const int64_t base = soa_stride(h->ntot);
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a), "hipEventCreate");
    HIP_TRY(hipEventCreate(&b), "hipEventCreate");
    float best = 1e30f;
    int64_t best_s = base;
    int rc = LBM_OK;
    for (int64_t pad : kStridePads) {
        h->stride = base + pad;
        rc = init_state(h, nullptr, nullptr);
        if (!rc) rc = enqueue_steps(h, 2);
        if (rc) break;
        hipError_t e = hipEventRecord(a, h->stream);
        if (e == hipSuccess) rc = enqueue_steps(h, 4);
        if (e == hipSuccess && !rc) e = hipEventRecord(b, h->stream);
        if (e == hipSuccess && !rc) e = hipEventSynchronize(b);
        float ms = 0.f;
        if (e == hipSuccess && !rc) e = hipEventElapsedTime(&ms, a, b);
        if (e != hipSuccess) rc = hip_fail(e, "stride trial");
        if (rc) break;
        if (std::getenv("LBM_VERBOSE"))
            std::fprintf(stderr, "lbm: stride %lld (pad %lld): %.3f ms per step\n", (long long)h->stride,
                         (long long)pad, ms / 4.0);
        if (ms < best) {
            best = ms;
            best_s = h->stride;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    h->stride = best_s;
    return rc;
}

static int autotune(lbm_handle* h)
{
    static const int cand[] = {64, 128, 256, 512, 1024};
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a), "hipEventCreate");
    HIP_TRY(hipEventCreate(&b), "hipEventCreate");
    float best = 1e30f;
    int best_b = 256;
    for (int c : cand) {
        if (c > max_step_block(h->d.lattice, h->d.collision, (int)elem_bytes(h->d.storage_dtype))) continue;
        h->block = c;
        int rc = enqueue_steps(h, 2);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(a, h->stream), "hipEventRecord");
        rc = enqueue_steps(h, 6);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(b, h->stream), "hipEventRecord");
        HIP_TRY(hipEventSynchronize(b), "hipEventSynchronize");
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
        if (ms < best) {
            best = ms;
            best_b = c;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    h->block = best_b;
    return LBM_OK;
}

// From the cell types in the flags: the fast-path hints, the fluid-cell
// count, the ascending list of fluid cells that need the general neighbour /
// bounce-back path, and the second stream that runs them.
static int build_tables(lbm_handle* h)
{
    const lbm_desc* d = &h->d;
    const uint32_t g = grid_for((uint64_t)h->ntot, 256);
    k_flag_hints<<<g, 256, 0, h->stream>>>(h->flags, d->nx, d->ny, d->nz, h->qlink ? 1 : 0);
    unsigned long long* cnt = (unsigned long long*)h->partial;
    k_zero_u64<<<1, 1, 0, h->stream>>>(cnt);
    k_count_fluid<<<g, 256, 0, h->stream>>>(h->flags, (uint64_t)h->ntot, cnt);
    unsigned long long nf = 0;
    HIP_TRY(hipMemcpyAsync(&nf, cnt, sizeof(nf), hipMemcpyDeviceToHost, h->stream), "flag set-up");
    HIP_TRY(hipStreamSynchronize(h->stream), "flag set-up");
    h->fluid = (int64_t)nf;

    std::vector<uint8_t> fl((size_t)h->ntot);
    HIP_TRY(hipMemcpy(fl.data(), h->flags, (size_t)h->ntot, hipMemcpyDeviceToHost), "flag read-back");
    const int64_t cpt = h->cpt;
    std::vector<uint32_t> slow, pull;
    for (int64_t g0 = 0; g0 < h->ntot; g0 += cpt) {
        // a group is fast when it is whole and every cell in it is a fast fluid cell
        bool fast = g0 + cpt <= h->ntot;
        // the vector kernels have no wall-plane path, so those cells are listed too
        const uint8_t off_path = cpt > 1 ? (FL_TYPE | FL_SLOW | FL_PLANE) : (FL_TYPE | FL_SLOW);
        for (int64_t i = g0; i < g0 + cpt && i < h->ntot; ++i)
            fast = fast && (fl[i] & off_path) == FL_FLUID;
        if (fast) continue;
        for (int64_t i = g0; i < g0 + cpt && i < h->ntot; ++i)
            if ((fl[i] & FL_TYPE) == FL_FLUID) {
                slow.push_back((uint32_t)i);
                if (cpt > 1 || !(fl[i] & FL_ZWRAP)) pull.push_back((uint32_t)i);
            }
    }
    if (h->slow_list) {
        HIP_TRY(hipFree(h->slow_list), "hipFree");
        h->slow_list = nullptr;
    }
    h->n_slow = (uint32_t)slow.size();
    h->n_slow_z = (uint32_t)pull.size();
    h->slow_list_z = nullptr;
    if (h->n_slow) {
        HIP_TRY(hipMalloc((void**)&h->slow_list, sizeof(uint32_t) * (slow.size() + pull.size())), "hipMalloc slow list");
        HIP_TRY(hipMemcpy(h->slow_list, slow.data(), sizeof(uint32_t) * slow.size(), hipMemcpyHostToDevice),
                "slow list");
        h->slow_list_z = h->slow_list + slow.size();
        if (!pull.empty())
            HIP_TRY(hipMemcpy(h->slow_list_z, pull.data(), sizeof(uint32_t) * pull.size(), hipMemcpyHostToDevice),
                    "slow list");
    }
    if (h->n_slow > 0 && !h->aux && !std::getenv("LBM_NO_OVERLAP") && (h->cpt > 1 || std::getenv("LBM_SPLIT_STEP"))) {
        HIP_TRY(hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking), "auxiliary stream");
        HIP_TRY(hipEventCreateWithFlags(&h->fork, hipEventDisableTiming), "auxiliary stream");
        HIP_TRY(hipEventCreateWithFlags(&h->join, hipEventDisableTiming), "auxiliary stream");
    }
    return LBM_OK;
}

// Caller buffers: 256-byte aligned and at least as large as
// lbm_required_bytes reports, checked before any device work.
static int check_caller_buffers(const lbm_desc* d)
{
    size_t req[3];
    if (int rc = lbm_required_bytes(d, req)) return rc;
    struct {
        const void* p;
        size_t have, need;
        const char* name;
    } const bufs[3] = {{d->pop, d->pop_bytes, req[0], "pop"},
                       {two_arrays(d->scheme) ? d->out : nullptr, d->out_bytes, req[1], "out"},
                       {d->flags, d->flags_bytes, req[2], "flags"}};
    for (const auto& b : bufs) {
        if (!b.p) continue;
        if ((uintptr_t)b.p % 256 != 0)
            return fail(LBM_EINVAL, std::string("caller buffer ") + b.name + " must be 256-byte aligned");
        if (b.have < b.need)
            return fail(LBM_EINVAL, std::string("caller buffer ") + b.name + " holds " + std::to_string(b.have) +
                                        " bytes, " + std::to_string(b.need) + " needed (lbm_required_bytes)");
    }
    return LBM_OK;
}

lbm_handle* lbm_create_ex(const lbm_desc* d)
{
    if (validate(d) || check_caller_buffers(d)) return nullptr;
    lbm_handle* h = new lbm_handle();
    h->d = *d;
    h->q = d->lattice;
    h->ntot = (int64_t)d->nx * d->ny * d->nz;
    // SoA: elements between streams; blocked: the padding cells before cell 0
    h->stride = d->layout == LBM_SOA ? soa_stride(h->ntot)
                                     : d->layout == LBM_BLOCKED ? blocked_pad(d->ny, d->nz) : h->ntot;
    h->stream = (hipStream_t)d->stream;
    h->launch = pick_tu(d->lattice, d->storage_dtype);
    h->block = std::min(d->block_size > 0 ? d->block_size : 256, max_step_block(d->lattice, d->collision, (int)elem_bytes(d->storage_dtype)));
    h->relax.omega = d->omega;
    h->relax.omega_m = d->collision == LBM_TRT ? trt_omega_minus(d->omega, d->trt_lambda) : d->omega;
    h->relax.omega_b = d->omega_bulk > 0.0 ? d->omega_bulk : d->omega;
    h->relax.omega3 = d->omega3 > 0.0 ? d->omega3 : 1.0;
    h->relax.omega4 = d->omega4 > 0.0 ? d->omega4 : 1.0;
    size_t req[3];
    lbm_required_bytes(d, req);
    h->pop_bytes = req[0];
    h->out_bytes = req[1];
    h->flag_bytes = req[2];

    auto bail = [&](int code, const std::string& msg) -> lbm_handle* {
        fail(code, msg);
        if (h->own_pop && h->pop_alloc) (void)hipFree(h->pop_alloc);
        if (h->own_out && h->out_alloc) (void)hipFree(h->out_alloc);
        if (h->own_flags && h->flags) (void)hipFree(h->flags);
        if (h->partial) (void)hipFree(h->partial);
        if (h->slow_list) (void)hipFree(h->slow_list);
        if (h->fork) (void)hipEventDestroy(h->fork);
        if (h->join) (void)hipEventDestroy(h->join);
        if (h->aux) (void)hipStreamDestroy(h->aux);
        delete h;
        return nullptr;
    };
    auto alloc = [&](void** p, size_t bytes, const char* what) -> bool {
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) {
            fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, std::string("hipMalloc ") + what + ": " + hipGetErrorString(e));
            *p = nullptr;
            return false;
        }
        return true;
    };
    if (d->pop) h->pop_alloc = d->pop;
    else if (alloc(&h->pop_alloc, h->pop_bytes, "pop")) h->own_pop = true;
    else return bail(LBM_ENOMEM, lbm_last_error());
    if (two_arrays(d->scheme)) {
        if (d->out) h->out_alloc = d->out;
        else if (alloc(&h->out_alloc, h->out_bytes, "out")) h->own_out = true;
        else return bail(LBM_ENOMEM, lbm_last_error());
    }
    if (d->flags) h->flags = (uint8_t*)d->flags;
    else if (alloc((void**)&h->flags, h->flag_bytes, "flags")) h->own_flags = true;
    else return bail(LBM_ENOMEM, lbm_last_error());
    {
        const size_t skip = d->layout == LBM_SOA ? (size_t)soa_halo(d->ny, d->nz) * elem_bytes(d->storage_dtype) : 0;
        h->pop = (char*)h->pop_alloc + skip;
        h->out = h->out_alloc ? (char*)h->out_alloc + skip : nullptr;
    }

    h->red_blocks = (int)grid_for((uint64_t)h->ntot, 256);
    if (!alloc((void**)&h->partial, sizeof(double) * (2 * (size_t)h->red_blocks + 2), "reduction"))
        return bail(LBM_ENOMEM, lbm_last_error());
    {
        hipError_t e = hipGetDevice(&h->device);
        if (e != hipSuccess) return bail(LBM_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
        if (int rc = scratch_address(h->device, &h->scratch)) return bail(rc, lbm_last_error());
    }

    // Flags: types, then fast-path hints, fluid count and edge-cell list.
    k_flag_types<<<grid_for((uint64_t)h->ntot, 256), 256, 0, h->stream>>>(h->flags, d->nx, d->ny, d->nz,
                                                                          d->geometry);
    h->cpt = d->layout == LBM_SOA ? cells_per_thread((int)elem_bytes(d->storage_dtype)) : 1;
    if (int rc = build_tables(h)) return bail(rc, lbm_last_error());
    h->use_graph = h->ntot <= kGraphCells && !std::getenv("LBM_NO_GRAPH");
    h->reverse_blocks = std::getenv("LBM_REVERSE_BLOCKS") != nullptr;
    if (const char* e = std::getenv("LBM_PULL_KERNEL"))
        h->pull_kernel = std::strcmp(e, "flag") == 0 ? 1 : (std::strcmp(e, "box") == 0 ? 2 : 0);
    if (const char* e = std::getenv("LBM_AA_KERNEL"))
        h->aa_kernel = std::strcmp(e, "flag") == 0 ? 1 : (std::strcmp(e, "box") == 0 ? 2 : 0);
    if (std::getenv("LBM_NO_RESIDENCY_CAP")) h->lds_override = true;  // lds_local = lds_neighbour = 0
    if (const char* e = std::getenv("LBM_STEP_LDS")) {  // "bytes" or "local,neighbour"
        unsigned a = 0, b = 0;
        const int got = std::sscanf(e, "%u,%u", &a, &b);
        h->lds_override = got >= 1;
        h->lds_local = got >= 1 ? std::min(a, 65536u) : 0;
        h->lds_neighbour = got >= 2 ? std::min(b, 65536u) : h->lds_local;
    }
    if (d->layout == LBM_SOA && h->ntot >= (int64_t(1) << 21) && !std::getenv("LBM_STRIDE_PAD") &&
        tune_stride(h))
        return bail(LBM_EDEVICE, lbm_last_error());
    if (init_state(h, nullptr, nullptr)) return bail(LBM_EDEVICE, lbm_last_error());
    if (d->block_size == -1) {
        if (autotune(h) || init_state(h, nullptr, nullptr)) return bail(LBM_EDEVICE, lbm_last_error());
    }
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return bail(LBM_EDEVICE, std::string("initialisation: ") + hipGetErrorString(e));
    return h;
}

lbm_handle* lbm_create(int lattice, int nx, int ny, int nz, int scheme, int collision, double omega, double u_lid,
                       int storage_dtype)
{
    lbm_desc d;
    lbm_desc_default(&d);
    d.lattice = lattice;
    d.nx = nx;
    d.ny = ny;
    d.nz = nz;
    d.scheme = scheme;
    d.collision = collision;
    d.omega = omega;
    d.lid_velocity[0] = u_lid;
    d.storage_dtype = storage_dtype;
    return lbm_create_ex(&d);
}

void lbm_destroy(lbm_handle* h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    if (h->aux) (void)hipStreamSynchronize(h->aux);
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    if (h->own_pop && h->pop_alloc) (void)hipFree(h->pop_alloc);
    if (h->own_out && h->out_alloc) (void)hipFree(h->out_alloc);
    if (h->own_flags && h->flags) (void)hipFree(h->flags);
    if (h->partial) (void)hipFree(h->partial);
    if (h->slow_list) (void)hipFree(h->slow_list);
    if (h->qlink) (void)hipFree(h->qlink);
    if (h->fork) (void)hipEventDestroy(h->fork);
    if (h->join) (void)hipEventDestroy(h->join);
    if (h->aux) (void)hipStreamDestroy(h->aux);
    delete h;
}

// Device staging for host pointers (ptr_kind = LBM_PTR_HOST).
struct Staging {
    void* dev = nullptr;
    ~Staging()
    {
        if (dev) (void)hipFree(dev);
    }
};

static int stage_in(lbm_handle* h, const void* src, size_t bytes, Staging& st, const void** dev)
{
    if (!src) {
        *dev = nullptr;
        return LBM_OK;
    }
    if (h->d.ptr_kind == LBM_PTR_DEVICE) {
        *dev = src;
        return LBM_OK;
    }
    HIP_TRY(hipMalloc(&st.dev, bytes), "hipMalloc staging");
    HIP_TRY(hipMemcpyAsync(st.dev, src, bytes, hipMemcpyHostToDevice, h->stream), "hipMemcpyAsync");
    *dev = st.dev;
    return LBM_OK;
}

static int stage_out_alloc(lbm_handle* h, void* dst, size_t bytes, Staging& st, void** dev)
{
    if (h->d.ptr_kind == LBM_PTR_DEVICE) {
        *dev = dst;
        return LBM_OK;
    }
    HIP_TRY(hipMalloc(&st.dev, bytes), "hipMalloc staging");
    *dev = st.dev;
    return LBM_OK;
}

static int stage_out_finish(lbm_handle* h, void* dst, size_t bytes, Staging& st)
{
    if (h->d.ptr_kind == LBM_PTR_HOST)
        HIP_TRY(hipMemcpyAsync(dst, st.dev, bytes, hipMemcpyDeviceToHost, h->stream), "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    return LBM_OK;
}

int lbm_init_equilibrium(lbm_handle* h, const double* rho, const double* u)
{
    if (!h) return fail(LBM_EINVAL, "null handle");
    Staging sr, su;
    const void *dr, *du;
    int rc = stage_in(h, rho, sizeof(double) * h->ntot, sr, &dr);
    if (!rc) rc = stage_in(h, u, sizeof(double) * 3 * h->ntot, su, &du);
    if (!rc) rc = init_state(h, (const double*)dr, (const double*)du);
    if (!rc && h->d.ptr_kind == LBM_PTR_HOST) HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    return rc;
}

int lbm_set_geometry(lbm_handle* h, const uint8_t* type, const double* wall_velocity, const double* wall_density)
{
    if (!h || !type) return fail(LBM_EINVAL, "null argument");
    Staging st, su, sr;
    const void *dt, *du, *dr;
    int rc = stage_in(h, type, (size_t)h->ntot, st, &dt);
    if (!rc) rc = stage_in(h, wall_velocity, sizeof(double) * 3 * h->ntot, su, &du);
    if (!rc) rc = stage_in(h, wall_density, sizeof(double) * h->ntot, sr, &dr);
    if (rc) return rc;
    const lbm_desc* d = &h->d;
    const int wrap = d->geometry == LBM_PERIODIC ? 7 : d->geometry == LBM_CHANNEL ? 3 : 0;
    const uint32_t g = grid_for((uint64_t)h->ntot, 256);
    unsigned long long* cnt = (unsigned long long*)h->partial;
    k_zero_u64<<<1, 1, 0, h->stream>>>(cnt);
    k_check_geometry<<<g, 256, 0, h->stream>>>((const uint8_t*)dt, (const double*)du, (const double*)dr, d->nx,
                                               d->ny, d->nz, wrap & 1, (wrap >> 1) & 1, (wrap >> 2) & 1, cnt);
    unsigned long long bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, cnt, sizeof(bad), hipMemcpyDeviceToHost, h->stream), "geometry check");
    HIP_TRY(hipStreamSynchronize(h->stream), "geometry check");
    if (bad)
        return fail(LBM_EINVAL, std::to_string(bad) + " cells break the geometry rules (types FLUID/WALL/LID/PRESSURE; "
                                "no fluid on a face that does not wrap; |u_w| < 0.4; 0 < rho_w < 10)");
    if (h->aux) HIP_TRY(hipStreamSynchronize(h->aux), "hipStreamSynchronize");
    if (h->graph) {  // its launches name the old edge-cell list
        HIP_TRY(hipGraphExecDestroy(h->graph), "hipGraphExecDestroy");
        h->graph = nullptr;
    }
    k_set_types<<<g, 256, 0, h->stream>>>((const uint8_t*)dt, h->flags, (uint64_t)h->ntot);
    rc = build_tables(h);
    if (rc) return rc;
    Launch L = h->base(OP_INIT);
    L.init.wall_u = (const double*)du;
    L.init.wall_rho = (const double*)dr;
    rc = run(h, L);
    if (rc) return rc;
    h->custom_walls = true;
    h->aa_phase = 0;
    h->steps = 0;
    h->first_nonfinite = -1;
    if (d->ptr_kind == LBM_PTR_HOST) HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    return LBM_OK;
}

int lbm_set_wall_distances(lbm_handle* h, const double* q)
{
    if (!h || !q) return fail(LBM_EINVAL, "null argument");
    Staging sq;
    const void* dq;
    const uint64_t n = (uint64_t)h->q * (uint64_t)h->ntot;
    int rc = stage_in(h, q, sizeof(double) * n, sq, &dq);
    if (rc) return rc;
    unsigned long long* cnt = (unsigned long long*)h->partial;
    k_zero_u64<<<1, 1, 0, h->stream>>>(cnt);
    k_zero_u64<<<1, 1, 0, h->stream>>>(cnt + 1);
    k_check_qlink<<<grid_for(n, 256), 256, 0, h->stream>>>((const double*)dq, n, cnt);
    unsigned long long c[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(c, cnt, sizeof(c), hipMemcpyDeviceToHost, h->stream), "wall distance check");
    HIP_TRY(hipStreamSynchronize(h->stream), "wall distance check");
    if (c[0]) return fail(LBM_EINVAL, std::to_string(c[0]) + " wall distances outside (0, 1]");
    if (c[1] && h->d.scheme != LBM_2POP_PULL)
        return fail(LBM_EUNSUPPORTED, "curved walls (distances other than 1/2) need the 2Pop pull scheme, whose "
                                      "gather reads every value the rule uses");
    if (h->aux) HIP_TRY(hipStreamSynchronize(h->aux), "hipStreamSynchronize");
    if (h->graph) {  // its launches name the old edge-cell list
        HIP_TRY(hipGraphExecDestroy(h->graph), "hipGraphExecDestroy");
        h->graph = nullptr;
    }
    if (!c[1]) {  // every wall half-way: the plain rule
        if (h->qlink) HIP_TRY(hipFree(h->qlink), "hipFree");
        h->qlink = nullptr;
    } else {
        if (!h->qlink) HIP_TRY(hipMalloc((void**)&h->qlink, sizeof(double) * n), "hipMalloc wall distances");
        HIP_TRY(hipMemcpyAsync(h->qlink, dq, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream),
                "wall distances");
    }
    k_clear_hints<<<grid_for((uint64_t)h->ntot, 256), 256, 0, h->stream>>>(h->flags, (uint64_t)h->ntot);
    rc = build_tables(h);  // curved links send every wall-adjacent fluid cell to the edge kernel
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    return LBM_OK;
}

static int invariants_raw(lbm_handle* h, double* mass, double* ke)
{
    Launch L = h->base(OP_INVARIANTS);
    L.block = 256;
    L.grid = (uint32_t)h->red_blocks;
    L.aa_odd = pending_gather(h);
    L.d0 = h->partial;
    int rc = run(h, L);
    if (rc) return rc;
    double* res = h->partial + 2 * (size_t)h->red_blocks;
    k_reduce_pairs<<<1, 256, 0, h->stream>>>(h->partial, h->red_blocks, res);
    double hr[2];
    HIP_TRY(hipMemcpyAsync(hr, res, sizeof(hr), hipMemcpyDeviceToHost, h->stream), "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    *mass = hr[0];
    *ke = hr[1];
    return LBM_OK;
}

int lbm_step(lbm_handle* h, int n)
{
    if (!h) return fail(LBM_EINVAL, "null handle");
    if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
    const int K = h->d.check_every;
    while (n > 0) {
        int chunk = n;
        if (K > 0) chunk = std::min<int64_t>(n, K - (h->steps % K));
        int rc = h->use_graph && K == 0 ? enqueue_steps_graph(h, chunk) : enqueue_steps(h, chunk);
        if (rc) return rc;
        n -= chunk;
        if (K > 0 && h->steps % K == 0) {
            double m, e;
            rc = invariants_raw(h, &m, &e);
            if (rc) return rc;
            if (!std::isfinite(m) || !std::isfinite(e)) {
                if (h->first_nonfinite < 0) h->first_nonfinite = h->steps;
                return fail(LBM_ENONFINITE, "non-finite mass or kinetic energy at step " + std::to_string(h->steps));
            }
        }
    }
    return LBM_OK;
}

int lbm_macroscopic(lbm_handle* h, double* rho, double* u)
{
    if (!h || !rho || !u) return fail(LBM_EINVAL, "null argument");
    Staging sr, su;
    void *dr, *du;
    int rc = stage_out_alloc(h, rho, sizeof(double) * h->ntot, sr, &dr);
    if (!rc) rc = stage_out_alloc(h, u, sizeof(double) * 3 * h->ntot, su, &du);
    if (rc) return rc;
    Launch L = h->base(OP_MACRO);
    L.aa_odd = pending_gather(h);
    L.d0 = (double*)dr;
    L.d1 = (double*)du;
    rc = run(h, L);
    if (!rc) rc = stage_out_finish(h, rho, sizeof(double) * h->ntot, sr);
    if (!rc) rc = stage_out_finish(h, u, sizeof(double) * 3 * h->ntot, su);
    return rc;
}

int lbm_get_populations(lbm_handle* h, double* f)
{
    if (!h || !f) return fail(LBM_EINVAL, "null argument");
    Staging s;
    void* df;
    const size_t bytes = sizeof(double) * h->q * h->ntot;
    int rc = stage_out_alloc(h, f, bytes, s, &df);
    if (rc) return rc;
    Launch L = h->base(OP_GET);
    L.aa_odd = pending_gather(h);
    L.d0 = (double*)df;
    rc = run(h, L);
    if (!rc) rc = stage_out_finish(h, f, bytes, s);
    return rc;
}

int lbm_get_populations_at(lbm_handle* h, const int64_t* cells, int n, double* f)
{
    if (!h || !cells || !f || n < 0) return fail(LBM_EINVAL, "bad argument");
    if (n == 0) return LBM_OK;
    if (h->d.ptr_kind == LBM_PTR_HOST)
        for (int j = 0; j < n; ++j)
            if (cells[j] < 0 || cells[j] >= h->ntot) return fail(LBM_EINVAL, "cell index out of range");
    Staging si, so;
    const void* dc;
    void* df;
    int rc = stage_in(h, cells, sizeof(int64_t) * n, si, &dc);
    if (!rc) rc = stage_out_alloc(h, f, sizeof(double) * n * h->q, so, &df);
    if (rc) return rc;
    Launch L = h->base(OP_GET_CELLS);
    L.aa_odd = pending_gather(h);
    L.cells = (const int64_t*)dc;
    L.d0 = (double*)df;
    L.n = n;
    L.grid = grid_for((uint64_t)n, L.block);
    rc = run(h, L);
    if (!rc) rc = stage_out_finish(h, f, sizeof(double) * n * h->q, so);
    return rc;
}

int lbm_set_populations(lbm_handle* h, const double* f)
{
    if (!h || !f) return fail(LBM_EINVAL, "null argument");
    Staging s;
    const void* df;
    int rc = stage_in(h, f, sizeof(double) * h->q * h->ntot, s, &df);
    if (rc) return rc;
    Launch L = h->base(OP_SET);
    L.c0 = (const double*)df;
    rc = run(h, L);
    if (rc) return rc;
    h->aa_phase = 0;
    h->steps = 0;
    h->first_nonfinite = -1;
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    return LBM_OK;
}

int lbm_get_flags(lbm_handle* h, uint8_t* flags)
{
    if (!h || !flags) return fail(LBM_EINVAL, "null argument");
    Staging s;
    void* df;
    int rc = stage_out_alloc(h, flags, (size_t)h->ntot, s, &df);
    if (rc) return rc;
    k_flag_types_only<<<grid_for((uint64_t)h->ntot, 256), 256, 0, h->stream>>>(h->flags, (uint8_t*)df, (uint64_t)h->ntot);
    HIP_TRY(hipGetLastError(), "kernel launch");
    return stage_out_finish(h, flags, (size_t)h->ntot, s);
}

int lbm_invariants(lbm_handle* h, double* mass, double* kinetic_energy)
{
    if (!h || !mass || !kinetic_energy) return fail(LBM_EINVAL, "null argument");
    return invariants_raw(h, mass, kinetic_energy);
}

// The kernels of lbm_invariants, with the partial sums in the GPU's copy of
// `scratch` (address looked up at creation) instead of the handle's buffer;
// no allocation, and no wait when the result is a device pointer.
int lbm_invariants_noalloc(lbm_handle* h, double* result)
{
    if (!h || !result) return fail(LBM_EINVAL, "null argument");
    if (h->ntot > kNoAllocMaxCells)
        return fail(LBM_EINVAL, "lbm_invariants_noalloc: " + std::to_string(h->ntot) +
                                    " cells exceed its scratch maximum of 2^25 cells (use lbm_invariants)");
    if (!h->scratch) return fail(LBM_EDEVICE, "lbm_invariants_noalloc: scratch address unknown");
    Launch L = h->base(OP_INVARIANTS);
    L.block = 256;
    L.grid = (uint32_t)h->red_blocks;
    L.aa_odd = pending_gather(h);
    L.d0 = h->scratch;
    int rc = run(h, L);
    if (rc) return rc;
    const bool host = h->d.ptr_kind == LBM_PTR_HOST;
    double* res = host ? h->scratch + 2 * (size_t)h->red_blocks : result;
    k_reduce_pairs<<<1, 256, 0, h->stream>>>(h->scratch, h->red_blocks, res);
    HIP_TRY(hipGetLastError(), "kernel launch");
    if (host) {
        HIP_TRY(hipMemcpyAsync(result, res, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream), "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    }
    return LBM_OK;
}

int lbm_neighbor_index(lbm_handle* h, const int64_t* cells, int n, int64_t* out)
{
    if (!h || !cells || !out || n < 0) return fail(LBM_EINVAL, "bad argument");
    if (n == 0) return LBM_OK;
    Staging si, so;
    const void* dc;
    void* dout;
    int rc = stage_in(h, cells, sizeof(int64_t) * n, si, &dc);
    if (!rc) rc = stage_out_alloc(h, out, sizeof(int64_t) * n * h->q, so, &dout);
    if (rc) return rc;
    if (h->d.ptr_kind == LBM_PTR_HOST) {
        for (int j = 0; j < n; ++j)
            if (cells[j] < 0 || cells[j] >= h->ntot) return fail(LBM_EINVAL, "cell index out of range");
    }
    Launch L = h->base(OP_NEIGHBORS);
    L.cells = (const int64_t*)dc;
    L.idx_out = (int64_t*)dout;
    L.n = n;
    L.grid = grid_for((uint64_t)n, L.block);
    rc = run(h, L);
    if (!rc) rc = stage_out_finish(h, out, sizeof(int64_t) * n * h->q, so);
    return rc;
}

int lbm_get_info(lbm_handle* h, lbm_info* info)
{
    if (!h || !info) return fail(LBM_EINVAL, "null argument");
    info->ntot = h->ntot;
    info->fluid_cells = h->fluid;
    info->pop_stride = h->stride;
    info->steps_done = h->steps;
    info->first_nonfinite = h->first_nonfinite;
    const int64_t s = (int64_t)elem_bytes(h->d.storage_dtype);
    info->bytes_per_update = h->d.scheme == LBM_SWAP ? 4 * h->q * s + 2 : 2 * h->q * s + 1;
    info->aa_phase = h->aa_phase;
    info->block_size = h->block;
    return LBM_OK;
}

int lbm_lattice(int lattice, int32_t* c, double* t, int32_t* opp)
{
    if (lattice != 19 && lattice != 27) return fail(LBM_EINVAL, "lattice must be 19 or 27");
    if (!c || !t || !opp) return fail(LBM_EINVAL, "null argument");
    auto fill = [&](auto s) {
        for (int k = 0; k < lattice; ++k) {
            for (int a = 0; a < 3; ++a) c[3 * k + a] = s.c[k][a];
            t[k] = s.t[k];
            opp[k] = s.opp[k];
        }
    };
    if (lattice == 19) fill(make_stencil<19>());
    else fill(make_stencil<27>());
    return LBM_OK;
}

int lbm_device_copy(void* dst, const void* src, size_t bytes, void* stream)
{
    if (!dst || !src || bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) % 16)
        return fail(LBM_EINVAL, "copy needs 16-byte aligned pointers and a multiple of 16 bytes");
    if (bytes == 0) return LBM_OK;
    const uint64_t n = bytes / 16;
    const uint32_t grid = (uint32_t)std::min<uint64_t>(grid_for(n, 256), 1u << 23);
    k_copy16<<<grid, 256, 0, (hipStream_t)stream>>>((uint4*)dst, (const uint4*)src, n);
    HIP_TRY(hipGetLastError(), "copy launch");
    return LBM_OK;
}

int lbm_pattern_copy(void* dst, const void* src, size_t n, size_t stride, int block_log2, int pattern, int vec,
                     int lds_bytes, int ny, int nz, void* stream)
{
    const bool blocked = block_log2 != 0;
    if (!dst || !src || n == 0 || n > 0xffffffffull || (block_log2 != 0 && block_log2 != 8 && block_log2 != 12) ||
        pattern < 0 || pattern > 2 || (vec != 1 && vec != 2) || (blocked && vec != 1) ||
        lds_bytes < 0 || lds_bytes > 65536 || (pattern > 0 && (ny < 1 || nz < 1)) || (int64_t)ny * nz > (1ll << 30) ||
        (!blocked && stride < n) || (blocked && n % ((size_t)1 << block_log2)) || n % (size_t)vec)
        return fail(LBM_EINVAL, "pattern copy: 1..2^32-1 values, layout SoA (stride >= n) or blocks of 2^8 / 2^12 "
                                "cells (n a multiple), pattern 0..2 with ny, nz >= 1 when shifted, 1 or 2 values "
                                "per lane (SoA), LDS 0..65536");
    const uint32_t grid = grid_for((uint64_t)n / vec, 256);
    hipStream_t st = (hipStream_t)stream;
    double* d = (double*)dst;
    const double* sp = (const double*)src;
    const uint32_t nn = (uint32_t)n, lds = (uint32_t)lds_bytes;
    auto go = [&](auto lbc) {
        constexpr int LB = decltype(lbc)::value;
        if (pattern == 0) launch_pattern<LB, 0>(vec, grid, lds, st, d, sp, stride, nn, ny, nz);
        else if (pattern == 1) launch_pattern<LB, 1>(vec, grid, lds, st, d, sp, stride, nn, ny, nz);
        else launch_pattern<LB, 2>(vec, grid, lds, st, d, sp, stride, nn, ny, nz);
    };
    if (block_log2 == 0) go(std::integral_constant<int, 0>{});
    else if (block_log2 == 8) go(std::integral_constant<int, 8>{});
    else go(std::integral_constant<int, 12>{});
    HIP_TRY(hipGetLastError(), "pattern copy launch");
    return LBM_OK;
}

int lbm_stream_copy(void* dst, const void* src, int nstreams, size_t n, size_t stride, int lds_bytes, int ny,
                    int nz, void* stream)
{
    if (!dst || !src || (nstreams != 19 && nstreams != 27) || n == 0 || n > 0xffffffffull || stride < n ||
        lds_bytes < 0 || lds_bytes > 65536 || ny < 0 || nz < 0 || (nz > 0 && ny < 1) ||
        (int64_t)ny * nz > (1ll << 30))
        return fail(LBM_EINVAL, "stream copy: 19 or 27 streams of 1..2^32-1 values, stride >= n, LDS 0..65536, "
                                "ny = nz = 0 or both >= 1");
    const uint32_t grid = grid_for((uint64_t)n, 256);
    if (nstreams == 19)
        k_copy_streams<19><<<grid, 256, (uint32_t)lds_bytes, (hipStream_t)stream>>>((double*)dst, (const double*)src,
                                                                                     stride, (uint32_t)n, ny, nz);
    else
        k_copy_streams<27><<<grid, 256, (uint32_t)lds_bytes, (hipStream_t)stream>>>((double*)dst, (const double*)src,
                                                                                     stride, (uint32_t)n, ny, nz);
    HIP_TRY(hipGetLastError(), "stream copy launch");
    return LBM_OK;
}

int lbm_sync(lbm_handle* h)
{
    if (!h) return fail(LBM_EINVAL, "null handle");
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    return LBM_OK;
}

}  // extern "C"
