// Types shared by the host runtime and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lbm {

// Flag byte: cell type in bits 0-1, fast-path hints in bits 6-7.
enum : uint8_t {
    FL_TYPE = 0x03,
    FL_FLUID = 0,
    FL_WALL = 1,
    FL_LID = 2,
    FL_PRESSURE = 3,  // pressure (density) wall: anti-bounce-back
    // Bits 2-4: wall plane of a fluid cell whose non-fluid neighbours are
    // exactly the nine on one side (1 x-1, 2 x+1, 3 y-1, 4 y+1, 5 z-1,
    // 6 z+1); such cells stay on the fast path.
    FL_PLANE_SHIFT = 2,
    FL_PLANE = 0x1C,
    // Fluid cell on a z face of a box that wraps in z, with x and y inside the
    // box and no solid neighbour: the fast paths of the pull and AA odd kernels
    // correct their z-wrapped accesses themselves (the other kinds list the
    // cell as a border cell).
    FL_ZWRAP = 0x20,
    FL_BORDER = 0x40,    // fluid cell on a box face: neighbours may wrap
    FL_NEARWALL = 0x80,  // fluid cell with any other pattern of non-fluid neighbours
    FL_SLOW = FL_BORDER | FL_NEARWALL,
};

enum Layout { LAYOUT_SOA = 0, LAYOUT_AOS = 1, LAYOUT_BLOCKED = 2 };
// Cells per block of the blocked layout (all Q streams of a block together).
#ifndef LBM_BLOCK_CELLS
#define LBM_BLOCK_CELLS 256
#endif
constexpr uint32_t kBlockCells = LBM_BLOCK_CELLS;
// KIND_PULL_Z, KIND_AA_ODD_Z: the fast parts of the pull and AA odd kernels
// for lattices with FL_ZWRAP cells.
enum Kind {
    KIND_2POP = 0, KIND_SWAP_COLLIDE = 1, KIND_SWAP_STREAM = 2, KIND_AA_EVEN = 3, KIND_AA_ODD = 4, KIND_PULL = 5,
    KIND_PULL_Z = 6, KIND_AA_ODD_Z = 7, KIND_PULL_BOX = 8, KIND_AA_ODD_BOX = 9, KIND_PULL_WRAP = 10,
    KIND_AA_ODD_WRAP = 11
};
enum Storage { STORE_F64 = 0, STORE_F32 = 1, STORE_F16 = 2 };

// Cells per thread of the fast step kernels: each lane updates this many
// consecutive cells and moves each population stream as one vector of
// LBM_VEC_BYTES (0: one cell per lane). Fluid cells of groups that are not
// entirely on the fast path go to the near-wall list.
#ifndef LBM_VEC_BYTES
#define LBM_VEC_BYTES 0
#endif
constexpr int cells_per_thread(int elem_bytes)
{
    return LBM_VEC_BYTES > elem_bytes ? LBM_VEC_BYTES / elem_bytes : 1;
}

struct StoreF64 {
    using T = double;
    using R = double;
    static constexpr bool shifted = false;
};
struct StoreF32 {
    using T = float;
    using R = float;
    static constexpr bool shifted = true;
};
struct StoreF16 {
    using T = _Float16;
    using R = float;
    static constexpr bool shifted = true;
};

// Momentum-exchange terms of a lid cell of the built-in geometries,
// w_k = -6 t_k c_k . u_lid with rho_w = 1 (Eq. storage2), computed once on
// the host and rounded to the storage type: every kernel that stores a lid
// cell's terms (initialisation, and the step kernels whose wall lanes write
// them back) takes them from this table, so they are the same bits wherever
// they are written, and the step kernels do no FP64 arithmetic for them.
struct LidTerms {
    double d[27];  // FP64 storage
    float f[27];   // FP32 and FP16 storage (the FP16 value held exactly in a float)
};

// One lattice as the kernels see it.
struct Field {
    void* pop;
    void* out;             // 2Pop destination (null otherwise)
    const uint8_t* flags;
    int64_t stride;        // SoA elements between populations
    uint32_t ntot;
    int nx, ny, nz;
    int reverse;           // visit cells in reverse block / list order (traversal-order tests)
    int custom_walls;      // wall terms set per cell by the caller (else: from type and lid)
    const double* qlink;   // curved walls: q[k][ntot], the wall's fraction of the link from a
                           //   fluid cell x to the wall cell x - c_k (null: all half-way)
    LidTerms lid;          // terms of lid cells (built-in geometries)
    uint64_t zrecip;       // ceil(2^64 / nz) (nz >= 2; else 0): floor(i / nz) = high word of i * zrecip
    uint64_t yrecip;       // ceil(2^64 / ny), the same for the row index (x ny + y) -> x
    int soa32;             // SoA whose streams and halo span under 4 GiB: 32-bit byte offsets suffice
    int run_rows;          // blocked layout with nz equal to the run: each row is one run
};

// Largest block of the step kernels: the moment-space models (model >= 4)
// and D3Q27 in FP64 need more registers per lane than 1024-thread blocks
// leave them (128 VGPRs). TRT and RR (models 1 and 3), which hold each
// population beside its opposite, spill at 128 VGPRs in the AA odd step in
// FP64 and on D3Q27; 512-thread blocks (256 VGPRs) remove the spills, which
// pays in FP64 (held to three waves per SIMD anyway) and in FP16 on D3Q27
// (+4 % on the 256^3 and 384^3 cavities). D3Q27 in FP32 keeps four waves
// with a few spilled registers: three waves without measured 2 % slower.
constexpr int max_step_block(int q, int model, int elem_bytes)
{
    if (model >= 4 || (q == 27 && elem_bytes == 8)) return 256;
    if ((model == 1 || model == 3) && (elem_bytes == 8 || (q == 27 && elem_bytes == 2))) return 512;
    return 1024;
}

// Waves per SIMD the registers of a fast step kernel must leave room for.
// FP64 kernels run at the two (AA odd and 2Pop pull: three) waves the
// residency cap below allows; the central-moment models on D3Q27 (AA odd) and D3Q19
// (CM, CHM, cumulant, AA odd) otherwise take one register too many for
// them (302 and 172-174 registers).
constexpr int min_step_waves(int q, int elem_bytes, int kind)
{
    if (elem_bytes != 8) return 1;
    return ((kind == 4 || kind == 5 || kind == 6 || kind == 7 || kind == 9 || kind == 10 || kind == 11) && q == 19)
               ? 3 : 2;
}

// Resident waves per SIMD the fast step kernels are held to (0: no limit),
// by bytes per stored value and kind. Measured on the 256^3 cavity: with FP64
// storage every wave keeps 38 streams of 512 B in flight, and two to three
// waves per SIMD move more bytes per second than the six the registers allow
// (AA: 15.2 -> 16.5 k MLUPS; 2Pop: 14.2 -> 15.2 k); FP32 gains with four on
// the kinds that touch only their own cell and 2Pop, and FP16 needs every
// wave it can get. Kinds: 0 2Pop, 1 swap collide, 2 swap stream, 3 AA even,
// 4 AA odd, 5 2Pop pull (FP64: 16.0 k at three to five waves, 15.7 k
// uncapped; FP32: 32.3 k uncapped, 31.4 k at four), 6 and 7 the z-wrap
// variants of 5 and 4, 8 the position-driven 2Pop pull of the built-in cavity
// (blocked layout, FP64: 18.2 k at two waves, 17.6 k at three, 17.5 k
// uncapped; FP32 and FP16 within 1 % of their best uncapped; the default FP64
// launch is blocks of 128, three per CU, set in run_kind), 9 its AA odd
// kind, 10 and 11 the position-driven pull and AA odd kinds of the periodic
// box.
inline int step_waves(int elem_bytes, int kind)
{
    if (kind == 8) return elem_bytes == 8 ? 2 : 0;
    if (kind == 9) return elem_bytes == 8 ? 2 : 0;  // FP64 SoA 16.8 k -> 17.0 k, blocked 17.1 k -> 17.3 k at 2
    if (kind == 10 || kind == 11) return elem_bytes == 8 ? 3 : 0;
    if (elem_bytes == 8) return (kind == 4 || kind >= 5) ? 3 : 2;
    if (elem_bytes == 4) return (kind == 4 || kind == 2 || kind >= 5) ? 0 : 4;
    return 0;
}

// Dynamic LDS per block that leaves room for the wanted number of resident
// waves per SIMD with blocks of the given size on a CU (160 KiB of LDS, at
// most 64 KiB per block, so at least two blocks). The size sits half a
// block's share below the limit, so the count holds whatever the allocation
// granularity. The kernels do not use it: it only caps residency.
inline uint32_t residency_lds_blocks(int blocks_per_cu)
{
    const uint32_t blocks = (uint32_t)(blocks_per_cu < 2 ? 2 : blocks_per_cu);
    const uint32_t v = (2u * 163840u / (2u * blocks + 1u)) / 1024u * 1024u;
    return v < 65536u ? v : 65536u;
}

inline uint32_t residency_lds(int waves_per_simd, int block)
{
    if (waves_per_simd <= 0) return 0;
    return residency_lds_blocks((waves_per_simd * 256) / (block < 64 ? 64 : block));
}

struct RelaxD {
    double omega, omega_m, omega_b, omega3, omega4;
};

struct InitArgs {
    const double* rho;     // device, may be null
    const double* u;       // device [3][ntot], may be null
    const double* wall_u;    // device [3][ntot]: per-cell wall velocity, may be null
    const double* wall_rho;  // device [ntot]: per-cell wall density, may be null
    int keep_walls;          // leave the stored terms of wall cells untouched
};

struct BatchCavity {
    Field F;
    RelaxD relax;
};

// A launch request handled by the kernel translation unit of (Q, storage).
enum Op { OP_STEP = 0, OP_GET = 1, OP_MACRO = 2, OP_SET = 3, OP_INIT = 4, OP_INVARIANTS = 5, OP_NEIGHBORS = 6,
          OP_STEP_BATCH = 7, OP_GET_CELLS = 8, OP_STEP_SLOW = 9,
          OP_STEP_ALL = 10, OP_STEP_BATCH_SLOW = 11 };

struct Launch {
    int op;
    int model, layout, kind;
    int aa_odd;
    int block;
    uint32_t grid;
    Field F;
    RelaxD relax;
    InitArgs init;
    double* d0;            // GET: f; MACRO: rho; INVARIANTS: partials
    double* d1;            // MACRO: u
    const double* c0;      // SET: f
    const int64_t* cells;  // NEIGHBORS
    int64_t* idx_out;
    int n;
    const BatchCavity* cav;  // STEP_BATCH, STEP_BATCH_SLOW
    const uint32_t* tiles;   // STEP_BATCH: (cavity << 16 | tile) per block
    uint32_t cpt;            // STEP_BATCH: runs of blockDim cells per tile
    int box;                 // STEP_BATCH: cells decided by position (box cavities), no edge part
    uint32_t xcd;            // STEP_BATCH: deal the tile table to the eight XCDs in contiguous parts
                             //   (grid a multiple of eight)
    const uint32_t* wave_cav;  // STEP_BATCH_SLOW: cavity of each wave of the edge-cell list
    const uint32_t* slow_list;  // STEP_SLOW, STEP: fluid cells off the fast path
    uint32_t n_slow;
    uint32_t edge_blocks;       // STEP: leading blocks that take slow_list (0: fast part only)
    uint32_t lds;          // STEP: dynamic LDS bytes per block (caps blocks per CU)
};

// Lid terms of a lattice of Q velocities stored in elements of elem_bytes
// (8, 4 or 2) for lid velocity u (host).
LidTerms lid_terms(int q, int elem_bytes, const double u[3]);

hipError_t launch_q19_f64(const Launch& L, hipStream_t s);
hipError_t launch_q19_f32(const Launch& L, hipStream_t s);
hipError_t launch_q19_f16(const Launch& L, hipStream_t s);
hipError_t launch_q27_f64(const Launch& L, hipStream_t s);
hipError_t launch_q27_f32(const Launch& L, hipStream_t s);
hipError_t launch_q27_f16(const Launch& L, hipStream_t s);
// Moment-space models (model >= NW4): step, init and batch launches.
hipError_t launch_q19_f64_mrt(const Launch& L, hipStream_t s);
hipError_t launch_q19_f32_mrt(const Launch& L, hipStream_t s);
hipError_t launch_q19_f16_mrt(const Launch& L, hipStream_t s);
hipError_t launch_q27_f64_mrt(const Launch& L, hipStream_t s);
hipError_t launch_q27_f32_mrt(const Launch& L, hipStream_t s);
hipError_t launch_q27_f16_mrt(const Launch& L, hipStream_t s);

}  // namespace lbm
