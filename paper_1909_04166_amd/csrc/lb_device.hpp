// lb_device.hpp -- device side of the fused stream-collide step for the coupled
// D2Q9 cascaded central-moment schemes (arXiv:1909.04166, Secs. 2-5), gfx950.
//
// Data layout (HBM): one lattice = two buffers (ping-pong) of the 18 stored
// values per node, f_0..f_8 then gbar_0..gbar_8, row-interleaved: value q of
// node (x, y) at element (18 y + q) nx + x (see row_stride).  A buffer holds the
// POST-COLLISION values of the previous step; the kernel pulls them
// (f_a(x) = f~_a(x - e_a)), so streaming costs nothing extra.
//
// One workgroup of TX lanes owns a strip of TX - 4 columns and a run of rows of
// one lattice (a work item); column slot t sits on column x0 - 2 + t, so the two
// halo columns on each side are ordinary lanes (see lane_slot for which lane holds
// which slot).  The workgroup marches upward one
// row per iteration:
//   A  every lane: pull f at the leading row L        -> phi(L)    (LDS ring)
//   B  lanes 1..w+2: pull gbar at row L-1             -> pbar(L-1) (LDS ring)
//   D  lanes 1..w+2: grad phi, n (or mu_phi) at row L-1           (LDS ring)
//   F  lanes 2..w+1: collide row L-2: div n (or grad mu), forces, u, p, both
//      collisions (the cascades in closed form), store the 18 post-collision values
// The pulled f and gbar of a lane stay in registers until their row is
// collided, so each stored value is read from HBM once per step (halo columns
// and the rows shared by neighbouring work items come from L2 / MALL).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lb_sched.hpp"

namespace cmlb {

// ------------------------------------------------------------------ storage

// `shifted`: whether the storage holds f_a - w_a shift (16-bit types only).
// st_sr(v, r): the stored value rounded stochastically with the random bits r
// (16-bit types; the wider types store v as it is).
struct StF64 {
    using T = double;
    using R = double;
    static constexpr int waves = 2;  // resident waves per SIMD the kernels are built for
    static constexpr bool shifted = false;
    static __device__ __forceinline__ R ld(T v) { return v; }
    static __device__ __forceinline__ T st(R v) { return v; }
    static __device__ __forceinline__ T st_sr(R v, uint32_t) { return v; }
};
struct StF32 {
    using T = float;
    using R = float;
    static constexpr int waves = 4;  // resident waves per SIMD the kernels are built for
    static constexpr bool shifted = false;
    static __device__ __forceinline__ R ld(T v) { return v; }
    static __device__ __forceinline__ T st(R v) { return v; }
    static __device__ __forceinline__ T st_sr(R v, uint32_t) { return v; }
};
// The gfx950 conversions with stochastic rounding (v_cvt_sr_f16_f32,
// v_cvt_sr_bf16_f32) take their random bits from the high 16 bits of r: the
// result is the representable neighbour above |v| with probability equal to the
// fraction of the gap that |v| has passed, so the stored value is unbiased.
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef short short2_t __attribute__((ext_vector_type(2)));
struct StF16 {
    using T = _Float16;
    using R = float;
    static constexpr int waves = 4;  // resident waves per SIMD the kernels are built for
    static constexpr bool shifted = true;
    static __device__ __forceinline__ R ld(T v) { return (float)v; }
    static __device__ __forceinline__ T st(R v) { return (_Float16)v; }  // round to nearest even
    static __device__ __forceinline__ T st_sr(R v, uint32_t r) {
        // the conversion writes the low half and keeps the high one, which is not
        // read: start from r's register rather than a zeroed one (no extra move)
        half2_t h = __builtin_bit_cast(half2_t, r);
        h = __builtin_amdgcn_cvt_sr_f16_f32(h, v, r, false);
        return h.x;
    }
};
struct StBF16 {
    using T = uint16_t;
    using R = float;
    static constexpr int waves = 4;  // resident waves per SIMD the kernels are built for
    static constexpr bool shifted = true;
    static __device__ __forceinline__ R ld(T v) { return __uint_as_float(((uint32_t)v) << 16); }
    static __device__ __forceinline__ T st(R v) {
        uint32_t u = __float_as_uint(v);
        if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))  // NaN stays NaN
            return (T)((u >> 16) | 0x0040u);
        u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
        return (T)(u >> 16);
    }
    static __device__ __forceinline__ T st_sr(R v, uint32_t r) {
        short2_t h = __builtin_bit_cast(short2_t, r);  // high half not read (see StF16)
        h = __builtin_amdgcn_cvt_sr_bf16_f32(h, v, r, false);
        return (T)(unsigned short)h.x;
    }
};

// ---------------------------------------------------------------- descriptors

// Per-lattice parameters, precomputed on the host.  Lives in device memory.
struct alignas(16) LatDesc {
    int32_t nx, ny;
    int32_t wall_y;     // walls at y = -1/2, ny - 1/2: 0 none (periodic), 1 halfway
                        // bounce-back, 2 halfway specular reflection (free slip)
    int32_t st_form;    // 0 geometric (+ Marangoni), 1 chemical potential
    int64_t plane;      // nodes per plane rounded up to 64 (buffer sizes, velocity planes)
    int32_t surf;       // kappa~(y): 0 linear, 1 Langmuir of an imposed linear psi(y)
    int32_t flow;       // 0 coupled, 1 phase field only under an imposed velocity
    int32_t wall_x;     // walls at x = -1/2, nx - 1/2: same codes as wall_y
    int32_t sround;     // 16-bit storage: 1 stochastic rounding of the stored values, 0 nearest even
    int32_t ntstore;    // 1: a row of one value plane is whole 128-byte lines (nx * size % 128 == 0)
    int32_t pad3;
    void* buf[2];       // 18 stored values per node each, row-interleaved (see row_stride)
    double* fields;     // FP64 output planes (phi, p, ux, uy or the 9 coupling planes)
    void* vel;          // imposed velocity: planes ux, uy in the compute type (flow 1)
    double* ktab;       // Langmuir law: kappa~(y) for y < ny, then d kappa~/dy (surf 1)
    uint32_t* tstep;    // tstep[p]: step count of the state in buf[p] (seeds the stochastic rounding)
    double rhoB, dRho;  // rho(phi) = rhoB + phi dRho
    double muB, dMu;    // mu(phi)  = muB + phi dMu
    double kt_a, kt_b;  // kappa~(y) = kt_a + kt_b y = 1.5 W sigma(y)
    double be_a, be_b;  // beta(y)  = 12 sigma(y) / W   (chemical-potential form)
    double ka_a, ka_b;  // kappa(y) = 1.5 W sigma(y)
    double four_W;      // 4 / W
    double M, omphi;    // mobility, first-order ACE rate 1 / (1/2 + 3 M)
    double gx, gy, rho_ref;
    double shift_f, shift_g;
    double kt0, lbeta, ps_a, ps_G;  // Langmuir: kappa~ = kt0 (1 + lbeta ln(1 - psi)), psi = ps_a + ps_G y
};


enum { MODE_STEP = 0, MODE_FIELDS = 1, MODE_COUPLING = 2 };
// Collision models of the coupled step: the cascaded pair, or the SRT pair of the
// stability comparison.
enum { COLL_CASCADED = 0, COLL_SRT = 1, COLL_PRINTED = 2 };
enum { PF_HOLD = 0, PF_PREFETCH = 1 };
enum { WALL_NONE = 0, WALL_BOUNCE = 1, WALL_SLIP = 2 };
// Kernel behind a step: coupled pair or phase field alone, cascaded or SRT.
enum { KIND_COUPLED_CASCADED = 0, KIND_COUPLED_SRT = 1, KIND_ACE_CASCADED = 2, KIND_ACE_SRT = 3,
       KIND_COUPLED_PRINTED = 4 };

// D2Q9 weights and velocities in the order 0 rest, 1 +x, 2 +y, 3 -x, 4 -y,
// 5 (+,+), 6 (-,+), 7 (-,-), 8 (+,-).
__device__ __forceinline__ double wgt(int a) {
    return a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
}

__device__ __forceinline__ int map_row(int L, int ny, int wall) {
    if (wall) return L < 0 ? -1 - L : (L >= ny ? 2 * ny - 1 - L : L);
    return L < 0 ? L + ny : (L >= ny ? L - ny : L);
}

// Element access through a uniform plane base and a 32-bit byte offset (every
// row block is < 4 GiB).  The pointers reach the kernels through the descriptor,
// so the compiler cannot see that they are global; naming the global address
// space here gives global (not flat) loads and stores with the base in scalar
// registers and a 32-bit per-lane offset, and keeps them off the LDS wait counter.
template <class T>
using gmem_t = __attribute__((address_space(1))) T;
// RAW: return the stored value as it is; the caller converts it later, so that a
// prefetch does not wait for its own load.
template <class ST, bool RAW = false>
__device__ __forceinline__ std::conditional_t<RAW, typename ST::T, typename ST::R> ldo(
    const typename ST::T* plane, uint32_t e) {
    using T = typename ST::T;
    const gmem_t<const char>* p = (const gmem_t<const char>*)plane;
    const T v = *(const gmem_t<const T>*)(p + e * (uint32_t)sizeof(T));
    if constexpr (RAW) return v; else return ST::ld(v);
}
// NT: nontemporal store (streamed past the caches; used where every stored row
// segment is whole cache lines, see lb_fused).
template <class ST, bool NT = false>
__device__ __forceinline__ void sto(typename ST::T* plane, uint32_t e, typename ST::R v) {
    using T = typename ST::T;
    gmem_t<char>* p = (gmem_t<char>*)plane;
    gmem_t<T>* q = (gmem_t<T>*)(p + e * (uint32_t)sizeof(T));
    if constexpr (NT) __builtin_nontemporal_store(ST::st(v), q);
    else *q = ST::st(v);
}

// The step kernels move 16- and 32-bit stored values through buffer resources: a
// descriptor in scalar registers holds the 64-bit base of one lattice row's block
// of values, the lane adds a 32-bit byte offset (its column) and the instruction a
// 32-bit uniform byte offset (the value's plane within the block, the same on
// every row).  No address then takes 64-bit arithmetic per access, which matters
// where the kernel is bound by instruction issue.  Kernels that wait on memory
// keep global accesses (a 64-bit scalar row base per access and a 32-bit lane
// offset): with buffer accesses the FP64 pair ran 8% slower and the FP32 phase
// field alone 4% slower.  kBufIO: the coupled pair in 16- and 32-bit storage;
// kBufIOAce: the phase field alone in 16-bit storage.
template <class ST>
constexpr bool kBufIO = sizeof(typename ST::T) < 8;
template <class ST>
constexpr bool kBufIOAce = sizeof(typename ST::T) < 4;
using rsrc_t = __amdgpu_buffer_rsrc_t;
typedef uint32_t u32x2 __attribute__((__vector_size__(8)));
__device__ __forceinline__ rsrc_t row_rsrc(const void* p) {
    // raw buffer (stride 0), every 32-bit offset in range, 32-bit data format
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, -1, 0x00020000);
}
template <class ST, bool RAW = false>
__device__ __forceinline__ std::conditional_t<RAW, typename ST::T, typename ST::R> ldb(rsrc_t r, uint32_t voff,
                                                                                        uint32_t soff) {
    using T = typename ST::T;
    T v;
    if constexpr (sizeof(T) == 2)
        v = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0));
    else if constexpr (sizeof(T) == 4)
        v = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
    else
        v = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
    if constexpr (RAW) return v; else return ST::ld(v);
}
// Cache-policy operand of the buffer stores: 2 is the nontemporal bit on gfx950.
template <bool NT>
constexpr int kStorePolicy = NT ? 2 : 0;
template <class ST, bool NT = false>
__device__ __forceinline__ void stb_raw(rsrc_t r, uint32_t voff, uint32_t soff, typename ST::T s) {
    using T = typename ST::T;
    if constexpr (sizeof(T) == 2)
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, s), r, (int)voff, (int)soff,
                                              kStorePolicy<NT>);
    else if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, s), r, (int)voff, (int)soff,
                                              kStorePolicy<NT>);
    else
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, s), r, (int)voff, (int)soff,
                                              kStorePolicy<NT>);
}
template <class ST, bool NT = false>
__device__ __forceinline__ void stb(rsrc_t r, uint32_t voff, uint32_t soff, typename ST::R v) {
    stb_raw<ST, NT>(r, voff, soff, ST::st(v));
}
// Stores values first..first+n-1 of row block `row` at column col.
template <class ST, int N, bool BUF, bool NT = false>
__device__ __forceinline__ void store_row(typename ST::T* row, int nx, int first, int col, const typename ST::R* v) {
    using T = typename ST::T;
    if constexpr (BUF) {
        const rsrc_t R = row_rsrc(row);
        const uint32_t P = (uint32_t)nx * (uint32_t)sizeof(T), b = (uint32_t)col * (uint32_t)sizeof(T);
#pragma unroll
        for (int a = 0; a < N; ++a) stb<ST, NT>(R, b, (uint32_t)(first + a) * P, v[a]);
    } else {
#pragma unroll
        for (int a = 0; a < N; ++a) sto<ST, NT>(row + (first + a) * nx, (uint32_t)col, v[a]);
    }
}

// Random bits of the stochastic rounding.  seed_step: an integer hash of the step
// count (two multiply-xorshift rounds, Wellons' lowbias32 constants; uniform over
// the launch); node_hash: that seed xor the node's index, times the golden-ratio
// constant, folded once (one multiply).  Stored value q of the node (0..8 f, 9..17
// gbar) then takes the low 32 bits of (h mod 2^24) x C_q, one full-rate 24-bit
// multiply per value, with 18 odd 24-bit multipliers C_q: over a 1024 x 512 grid
// the top 16 bits of each product (the bits the conversions use) are uniform to
// 1e-3, and their correlation across q, between neighbouring nodes and between
// consecutive steps stays at the sampling noise (below 0.006).  The bits depend on
// the step and the node only, so every schedule stores the same values.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
__device__ __forceinline__ uint32_t seed_step(uint32_t t) { return mix32(t * 0x9e3779b9u + 0x7f4a7c15u); }
__device__ __forceinline__ uint32_t node_hash(uint32_t seed, int x, int y) {
    uint32_t h = (seed ^ ((uint32_t)y * 0x85ebca6bu + (uint32_t)x)) * 0x9e3779b1u;
    return h ^ (h >> 16);
}
constexpr uint32_t kSRMul[18] = {0xa58a9du, 0xfb4889u, 0x987a27u, 0xb9e081u, 0xe3f42fu, 0xe90a67u,
                                 0xfe72f1u, 0x8a7dabu, 0x937427u, 0x99dcefu, 0xae49f3u, 0xbe1d1bu,
                                 0xd0335du, 0xfcb1d9u, 0xdf8a85u, 0xd8aadfu, 0xbd9efbu, 0x8eca35u};

// As store_row, rounding value first + a stochastically with the bits of node hash h.
template <class ST, int N, bool BUF, bool NT = false>
__device__ __forceinline__ void store_row_sr(typename ST::T* row, int nx, int first, int col,
                                             const typename ST::R* v, uint32_t h) {
    using T = typename ST::T;
    gmem_t<char>* base = (gmem_t<char>*)row;
    const uint32_t P = (uint32_t)nx * (uint32_t)sizeof(T), b = (uint32_t)col * (uint32_t)sizeof(T);
    const uint32_t h24 = h & 0xffffffu;
#pragma unroll
    for (int a = 0; a < N; ++a) {
        const T s = ST::st_sr(v[a], h24 * kSRMul[first + a]);
        if constexpr (BUF) {
            stb_raw<ST, NT>(row_rsrc(row), b, (uint32_t)(first + a) * P, s);
        } else {
            gmem_t<T>* q = (gmem_t<T>*)(base + (uint32_t)(first + a) * P + b);
            if constexpr (NT) __builtin_nontemporal_store(s, q);
            else *q = s;
        }
    }
}

// The nine collided values of a node from value `first` on: rounded
// stochastically with node hash h when sr (16-bit storage), else to nearest;
// nontemporal stores when NT.
template <class ST, bool BUF, bool NT>
__device__ __forceinline__ void store_collided(bool sr, typename ST::T* row, int nx, int first, int col,
                                               const typename ST::R* v, uint32_t h) {
    if constexpr (ST::shifted) {
        if (sr) {
            store_row_sr<ST, 9, BUF, NT>(row, nx, first, col, v, h);
            return;
        }
    }
    store_row<ST, 9, BUF, NT>(row, nx, first, col, v);
}

// Buffer layout: the 18 stored values of a lattice are row-interleaved, value q
// (0..8 f, 9..17 gbar) of node (x, y) at element (18 y + q) nx + x.  The nine f
// (or gbar) rows of one lattice row form one contiguous block, so a workgroup
// streams three blocks per row instead of eighteen scattered planes.  Row bases
// are formed in 64-bit uniform arithmetic, lane offsets within a block in 32 bits.
__device__ __forceinline__ int64_t row_stride(int nx) { return 18 * (int64_t)nx; }
// Row block r (0 <= r < ny) of a buffer, with the element offset formed by one
// 32 x 32 -> 64-bit multiply (18 nx fits 32 bits) instead of a 64 x 64 one.
template <class T>
__device__ __forceinline__ T* row_at(T* base, int r, int nx) {
    return base + (uint64_t)(uint32_t)r * (uint32_t)row_stride(nx);
}

// Pull the nine stored values arriving at (x, r): f_a(x, r) = f~_a(x - e_a).  A source
// beyond a halfway wall is replaced by the opposite direction at the same node
// (bounce-back), or by the y-mirrored direction at the node the particle left,
// x - e_ax (specular reflection).  base points at value 0 of row 0 of the group
// (f or gbar); xm, xp are the periodic neighbours of x.  BUF: buffer accesses.
template <class ST, bool BUF, bool RAW = false>
__device__ __forceinline__ void pull9(const typename ST::T* __restrict__ base, int nx, int ny,
                                      int wall, int wallx, int x, int xm, int xp, int r,
                                      std::conditional_t<RAW, typename ST::T, typename ST::R> out[9]) {
    using T = typename ST::T;
    const bool bot = wall && r == 0;       // sources of 2, 5, 6 lie below the wall
    const bool top = wall && r == ny - 1;  // sources of 4, 7, 8 lie above the wall
    const bool slip = wall == WALL_SLIP;
    const int rb = r == 0 ? ny - 1 : r - 1;
    const int rt = r == ny - 1 ? 0 : r + 1;
    const T* ro = row_at(base, r, nx);
    const T* rbp = row_at(base, rb, nx);  // row below (periodic image)
    const T* rtp = row_at(base, rt, nx);  // row above
    // On the rows next to a y wall every source is selected (uniform value block
    // and row, per-lane column), so that the nine loads issue together.
    const T* sb = bot ? ro : rbp;
    const T* st = top ? ro : rtp;
    const uint32_t P = (uint32_t)nx * (uint32_t)sizeof(T);  // bytes between value planes
    // value `plane` of row block `row` at column `col`
    auto ld = [&](const T* row, uint32_t plane, int col) {
        if constexpr (BUF)
            return ldb<ST, RAW>(row_rsrc(row), (uint32_t)col * (uint32_t)sizeof(T), plane * P);
        else
            return ldo<ST, RAW>(row + (int)plane * nx, (uint32_t)col);
    };
    out[0] = ld(ro, 0, x);
    out[1] = ld(ro, 1, xm);
    out[3] = ld(ro, 3, xp);
    if (!bot && !top) {
        // every row but the two next to a y wall (uniform branch): the plain pull
        out[2] = ld(rbp, 2, x);
        out[5] = ld(rbp, 5, xm);
        out[6] = ld(rbp, 6, xp);
        out[4] = ld(rtp, 4, x);
        out[7] = ld(rtp, 7, xp);
        out[8] = ld(rtp, 8, xm);
    } else {
        const uint32_t p2 = bot ? 4 : 2, p5 = bot ? (slip ? 8 : 7) : 5, p6 = bot ? (slip ? 7 : 8) : 6;
        const uint32_t p4 = top ? 2 : 4, p7 = top ? (slip ? 6 : 5) : 7, p8 = top ? (slip ? 5 : 6) : 8;
        const int x5 = (bot && !slip) ? x : xm, x6 = (bot && !slip) ? x : xp;
        const int x7 = (top && !slip) ? x : xp, x8 = (top && !slip) ? x : xm;
        out[2] = ld(sb, p2, x);
        out[5] = ld(sb, p5, x5);
        out[6] = ld(sb, p6, x6);
        out[4] = ld(st, p4, x);
        out[7] = ld(st, p7, x7);
        out[8] = ld(st, p8, x8);
    }
    if (wallx) {
        // Lanes on the first or last column replace what arrived from beyond an x
        // wall: bounce-back (opposite direction, same node), or specular reflection
        // (x-mirrored direction leaving the node of the same column one row over);
        // beyond an x and a y wall at once, bounce-back.
        const bool sx = wallx == WALL_SLIP;
        if (x == 0) {
            out[1] = ld(ro, 3, x);
            out[5] = (sx && !bot) ? ld(rbp, 6, x) : ld(ro, 7, x);
            out[8] = (sx && !top) ? ld(rtp, 7, x) : ld(ro, 6, x);
        }
        if (x == nx - 1) {
            out[3] = ld(ro, 1, x);
            out[6] = (sx && !bot) ? ld(rbp, 5, x) : ld(ro, 8, x);
            out[7] = (sx && !top) ? ld(rtp, 8, x) : ld(ro, 5, x);
        }
    }
}

// Marks the lane's column indices as redefined inside the row loop (an empty asm
// statement: no instruction).  Otherwise the compiler hoists their widened byte
// offsets out of the loop as 64-bit values and forms every address with a 64-bit
// vector add; redefined in the loop, each access becomes a global load or store
// with the 64-bit row base in scalar registers and a 32-bit lane offset.
__device__ __forceinline__ void lane_columns_in_loop(int& xc, int& xm, int& xp) {
    asm volatile("" : "+v"(xc), "+v"(xm), "+v"(xp));
}

// Column slot of a lane in a TX-lane workgroup: slots 0, 1 and TX-2, TX-1 hold the
// halo columns, slots 2..TX-3 the strip (slot s sits on column x0 - 2 + s).  Lanes
// 0..TX-5 take the strip (slot = lane + 2) and the last four lanes the halo, so with
// TX - 4 a multiple of 64 every wave but the last starts its loads and stores of the
// strip on a cache-line boundary (x0 is then a multiple of 64).
template <int TX>
__device__ __forceinline__ int lane_slot(int lane) {
    return lane < TX - 4 ? lane + 2 : (lane < TX - 2 ? lane - (TX - 4) : lane);
}

// The sum of the nine values, in pairs that the moments below share (the
// compiler computes each pair once).
template <class R>
__device__ __forceinline__ R sum9(const R v[9]) {
    return v[0] + (((v[1] + v[3]) + (v[2] + v[4])) + ((v[5] + v[6]) + (v[7] + v[8])));
}

// What the cascaded collisions read of the pulled values (see ace_collide and
// hydro_collide): of f the sum of the stored values and the first moments k10,
// k01; of gbar the first moments j and the two shear differences of its raw
// second moments, (g1 + g3) - (g2 + g4) = eta_20 - eta_02 and (g5 - g6) + (g7 - g8)
// = eta_11.  The sum of gbar (pbar) goes to the LDS ring when the row is pulled.
// The row pipeline of the fused step holds these instead of the nine values (the
// SRT collisions read every value and hold them all).
template <class R>
struct FMom {
    R tot, k10, k01;
};
template <class R>
struct GMom {
    R jx, jy, nd, xd;
};
template <class R>
struct Vals9 {
    R v[9];
};
// First moments; (v8 - v7) is taken as -(v7 - v8), exactly the same value, so that
// the difference is shared with the shear moment of gbar.
template <class R>
__device__ __forceinline__ R first_x(const R v[9]) {
    return ((v[1] - v[3]) + (v[5] - v[6])) - (v[7] - v[8]);
}
template <class R>
__device__ __forceinline__ R first_y(const R v[9]) {
    return ((v[2] - v[4]) + (v[5] + v[6])) - (v[7] + v[8]);
}
template <class R>
__device__ __forceinline__ void hold(FMom<R>& h, const R v[9]) {
    h.tot = sum9(v);
    h.k10 = first_x(v);
    h.k01 = first_y(v);
}
template <class R>
__device__ __forceinline__ void hold(GMom<R>& h, const R v[9]) {
    h.jx = first_x(v);
    h.jy = first_y(v);
    h.nd = (v[1] + v[3]) - (v[2] + v[4]);
    h.xd = (v[5] - v[6]) + (v[7] - v[8]);
}
template <class R>
__device__ __forceinline__ void hold(Vals9<R>& h, const R v[9]) {
#pragma unroll
    for (int a = 0; a < 9; ++a) h.v[a] = v[a];
}
template <class R>
__device__ __forceinline__ R held_sum(const FMom<R>& h) { return h.tot; }
template <class R>
__device__ __forceinline__ R held_sum(const Vals9<R>& h) { return sum9(h.v); }
template <class R>
__device__ __forceinline__ void held_first(const GMom<R>& h, R& jx, R& jy) { jx = h.jx; jy = h.jy; }
template <class R>
__device__ __forceinline__ void held_first(const Vals9<R>& h, R& jx, R& jy) {
    jx = first_x(h.v);
    jy = first_y(h.v);
}

// Isotropic D2Q9 gradient (1/c^2) sum_a w_a e_a q(x + e_a) from a 3x3 patch:
// rows s (y-1), m (y), n (y+1); columns c-1, c, c+1.
template <class R>
__device__ __forceinline__ void grad3x3(const R* s, const R* m, const R* n, int c, R& gx, R& gy) {
    const R k1 = R(1.0 / 3.0), k2 = R(1.0 / 12.0);
    gx = k1 * (m[c + 1] - m[c - 1]) + k2 * ((n[c + 1] - n[c - 1]) + (s[c + 1] - s[c - 1]));
    gy = k1 * (n[c] - s[c]) + k2 * ((n[c + 1] + n[c - 1]) - (s[c + 1] + s[c - 1]));
}

// Isotropic D2Q9 Laplacian (2/c^2) sum_a w_a (q(x + e_a) - q(x)).
template <class R>
__device__ __forceinline__ R lap3x3(const R* s, const R* m, const R* n, int c) {
    const R axis = (m[c + 1] + m[c - 1]) + (n[c] + s[c]);
    const R diag = (n[c + 1] + n[c - 1]) + (s[c + 1] + s[c - 1]);
    return R(2.0 / 3.0) * axis + R(1.0 / 6.0) * diag - R(10.0 / 3.0) * m[c];
}

// ------------------------------------------------------ per-node physics

// Per-lattice constants in the compute type, loaded once per work item.
template <class R>
struct KConst {
    R rhoB, dRho, muB, dMu, kt_a, kt_b, be_a, be_b, ka_a, ka_b, four_W, M, omphi, gx, gy, rho_ref,
        shf, shg, c2dr;
};

template <class R>
__device__ __forceinline__ KConst<R> load_const(const LatDesc& D) {
    KConst<R> k;
    k.rhoB = R(D.rhoB); k.dRho = R(D.dRho); k.muB = R(D.muB); k.dMu = R(D.dMu);
    k.kt_a = R(D.kt_a); k.kt_b = R(D.kt_b); k.be_a = R(D.be_a); k.be_b = R(D.be_b);
    k.ka_a = R(D.ka_a); k.ka_b = R(D.ka_b); k.four_W = R(D.four_W); k.M = R(D.M);
    k.omphi = R(D.omphi); k.gx = R(D.gx); k.gy = R(D.gy); k.rho_ref = R(D.rho_ref);
    k.shf = R(D.shift_f); k.shg = R(D.shift_g); k.c2dr = R(D.dRho * (1.0 / 3.0));
    return k;
}

// Reciprocal: correctly rounded in FP64, hardware v_rcp_f32 (1 ulp) in FP32.
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Unit normal from a gradient; zero where |grad phi| < 1e-12.
__device__ __forceinline__ void unit_normal(double gx, double gy, double m2, double& nx, double& ny) {
    const double m = sqrt(m2);
    nx = 0.0; ny = 0.0;
    if (!(m < 1e-12)) { const double im = 1.0 / m; nx = gx * im; ny = gy * im; }
}
__device__ __forceinline__ void unit_normal(float gx, float gy, float m2, float& nx, float& ny) {
    nx = 0.0f; ny = 0.0f;
    if (!(m2 < 1e-24f)) { const float im = __builtin_amdgcn_rsqf(m2); nx = gx * im; ny = gy * im; }
}

template <class R>
struct NodeIn {
    R phi, pbar;
    R dphx, dphy, m2, nx, ny;  // grad phi, |grad phi|^2, unit normal (0 where undefined)
    R divn;                    // div n (geometric form)
    R dmux, dmuy;              // grad mu_phi (chemical-potential form)
    R dpx, dpy;                // grad pbar
    R kt, dkt;                 // kappa~ at the node's row and d kappa~ / dy (geometric form)
};

// kappa~ and d kappa~/dy of row y: the linear law kt_a + kt_b y, or the Langmuir
// law read from the per-row table (computed once per lattice by k_kappa_table;
// evaluating the logarithm here would cost the FP64 kernel half its occupancy).
template <class R>
__device__ __forceinline__ void row_kappa(const KConst<R>& K, const double* ktab, int ny, int y, R& kt,
                                          R& dkt) {
    if (ktab) {
        kt = R(ktab[y]);
        dkt = R(ktab[ny + y]);
    } else {
        kt = K.kt_a + K.kt_b * R(y);
        dkt = K.kt_b;
    }
}

template <class R>
struct NodeOut {
    R rho, omv, ux, uy, p, Ftx, Fty, Fpx, Fpy;
    R jx, jy;  // first moments of the pre-collision gbar
};

// Properties, forces, velocity and pressure of one node (Eqs.
// sfluidpropertiesinterpolation, surfacetensiongeometricsurfactantsxcomp/ycomp,
// surfacetensionthermodynamic, netgradientpressureforce, hydrodynamicfields,
// fluidviscosity).
template <class R>
__device__ __forceinline__ NodeOut<R> node_macro(const KConst<R>& K, int chem, const NodeIn<R>& in, R jx,
                                                 R jy) {
    NodeOut<R> o;
    const R rho = K.rhoB + in.phi * K.dRho;
    const R mu = K.muB + in.phi * K.dMu;
    const R den = R(0.5) * rho + R(3) * mu;  // rho (1/omega_nu) with nu = mu / rho
    const R rr = rcp(rho * den);
    const R inv_rho = den * rr;
    o.rho = rho;
    o.omv = rho * rho * rr;
    R Fsx, Fsy;
    if (!chem) {
        const R a = in.m2 * in.kt * in.divn;
        const R b = in.m2 * in.dkt;
        Fsx = -a * in.nx - b * in.nx * in.ny;
        Fsy = -a * in.ny + b * (R(1) - in.ny * in.ny);
    } else {
        Fsx = -in.phi * in.dmux;
        Fsy = -in.phi * in.dmuy;
    }
    const R bf = rho - K.rho_ref;
    o.Ftx = Fsx + bf * K.gx;
    o.Fty = Fsy + bf * K.gy;
    o.jx = jx;
    o.jy = jy;
    o.ux = (R(3) * jx + R(0.5) * o.Ftx) * inv_rho;
    o.uy = (R(3) * jy + R(0.5) * o.Fty) * inv_rho;
    o.Fpx = -in.dpx + K.c2dr * in.dphx;
    o.Fpy = -in.dpy + K.c2dr * in.dphy;
    o.p = in.pbar + R(0.5) * (o.Fpx * o.ux + o.Fpy * o.uy);
    return o;
}

// Stored values of shifted 16-bit storage are s_a = f_a - w_a sh.  The shift's raw
// moments are (sh, 0, 0, sh/3, sh/3, 0, 0, 0, sh/9), and its first and shear
// moments vanish, so the collisions read those moments from s directly and
// subtract the shift's moments from what they store.  With SH false no
// instruction is spent on it.

// Pressure-based cascaded collision with its cumulative source (Sec. 4), with
// omega_0..3 = omega_6..8 = 1 and omega_4 = omega_5 = omv.  SOLVED (the
// collision of the cascaded pair): h_3..h_8 solve the relaxation conditions as
// stated; otherwise (the printed option) their printed closed forms are used.
//
// Written out with the printed closed forms, the cascade (moment changes h_0..h_8
// of Eq. cascadedcollisionoperator plus the source K^{-1}(I - Lambda/2) K S) leaves
// post-collision raw moments that depend on the incoming values only through
// pbar, j and the two shear non-equilibria
//   N = (eta_20 - eta_02) - c^2 rho (ux^2 - uy^2),   X = eta_11 - c^2 rho ux uy,
// each relaxed by (1 - omv):
//   m00 = pbar + G                                   (G = F_p . u)
//   m10 = j_x + c^2 F_tx,  m01 = j_y + c^2 F_ty
//   m20 + m02 = 2 c^2 p + c^2 rho |u|^2 + 4/3 G + c^2 F_t . u
//   m20 - m02 = c^2 rho (ux^2 - uy^2) + (1 - omv) N + (1 - omv/2)(s20 - s02)
//   m11 = c^2 rho ux uy + (1 - omv) X + (1 - omv/2) s11
//   m21 = c^2 rho uy (c^2 + ux^2) + c^4 F_ty + (1 - omv)(uy N / 2 + 2 ux X)
//   m12 = c^2 rho ux (c^2 + uy^2) + c^4 F_tx + (1 - omv)(-ux N / 2 + 2 uy X)
//   m22 = c^4 p + c^4 rho |u|^2 + c^2 rho ux^2 uy^2 + 2 c^4 G
//         + (1 - omv)(-(ux^2 - uy^2) N / 2 + 4 ux uy X)
// with s20, s02, s11 the second-order raw source moments.  These equal the
// cascade term by term (a symbolic identity in the incoming moments, u, p, rho and
// the forces); evaluating them and inverting the moment map costs about 100
// operations instead of 150 and never forms the O(rho) terms of psi = p - c^2 rho
// that cancel in the cascade.  Shifted storage subtracts the raw moments of w sh
// (sh, 0, 0, sh/3, sh/3, 0, 0, 0, sh/9); N, X and j are shift-free.
//
// SOLVED: the relaxation conditions of the cascaded collision (Sec. 4) solved as
// stated, with the central moments of the incoming gbar itself (zeroth moment
// pbar, first j) and the source-driven h_0..h_2 carried into the higher central
// moments, instead of the printed closed forms of h_3..h_8 (which leave those two
// effects out).  The post-collision raw moments are then the ones above with the
// shear non-equilibria taken about u,
//   N' = N + c^2 (F_tx ux - F_ty uy) - (ux^2 - uy^2) G / 2,
//   X' = X + c^2 (F_tx uy + F_ty ux) / 2 - ux uy G / 2,
// and without the force terms (2/3) G of m20 + m02, c^4 F_ty of m21, c^4 F_tx of
// m12 and 2 c^4 G of m22 (a symbolic identity with the numerical solve of the same
// conditions; it costs the printed form's operations).
template <class R, bool SH = false, bool SOLVED = false>
__device__ __forceinline__ void hydro_collide(R g[9], const NodeOut<R>& o, R nd, R xd, R sh = R(0)) {
    const R ux = o.ux, uy = o.uy, ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy;
    const R third = R(1.0 / 3.0), ninth = R(1.0 / 9.0);
    const R rc2 = o.rho * third;
    const R Gam = o.Fpx * ux + o.Fpy * uy;
    const R Sx = o.Ftx + o.Fpx, Sy = o.Fty + o.Fpy;
    const R hw = R(1) - R(0.5) * o.omv;
    const R om1 = R(1) - o.omv;
    R nraw = nd - rc2 * (ux2 - uy2);  // N
    R xraw = xd - rc2 * uxy;          // X
    if constexpr (SOLVED) {  // N', X': the non-equilibria about u
        nraw += third * (o.Ftx * ux - o.Fty * uy) - R(0.5) * (ux2 - uy2) * Gam;
        xraw += R(1.0 / 6.0) * (o.Ftx * uy + o.Fty * ux) - R(0.5) * uxy * Gam;
    }
    const R nn = om1 * nraw;
    const R xx = om1 * xraw;
    const R m00 = o.p + R(0.5) * Gam - (SH ? sh : R(0));
    const R m10 = o.jx + third * o.Ftx, m01 = o.jy + third * o.Fty;
    const R T = R(2.0 / 3.0) * o.p + rc2 * (ux2 + uy2) + (SOLVED ? R(2.0 / 3.0) : R(4.0 / 3.0)) * Gam +
                third * (o.Ftx * ux + o.Fty * uy) - (SH ? R(2.0 / 3.0) * sh : R(0));
    const R D = rc2 * (ux2 - uy2) + nn + hw * R(2.0 / 3.0) * (Sx * ux - Sy * uy);
    const R m11 = rc2 * uxy + xx + hw * third * (Sx * uy + Sy * ux);
    const R m21 = rc2 * uy * (third + ux2) + (SOLVED ? R(0) : ninth * o.Fty) + R(0.5) * uy * nn + R(2) * ux * xx;
    const R m12 = rc2 * ux * (third + uy2) + (SOLVED ? R(0) : ninth * o.Ftx) - R(0.5) * ux * nn + R(2) * uy * xx;
    const R m22 = ninth * o.p + o.rho * (ninth * (ux2 + uy2) + third * ux2 * uy2) +
                  (SOLVED ? R(0) : R(2.0 / 9.0) * Gam) - R(0.5) * (ux2 - uy2) * nn + R(4) * uxy * xx -
                  (SH ? ninth * sh : R(0));
    // inverse of the moment map (m20 = (T + D)/2, m02 = (T - D)/2)
    const R a = R(0.5) * (T + D) - m22, b = m10 - m12;
    const R c = R(0.5) * (T - D) - m22, d = m01 - m21;
    const R u1 = m22 + m11, u2 = m22 - m11, v1 = m21 + m12, v2 = m21 - m12;
    g[0] = m00 - T + m22;
    g[1] = R(0.5) * (a + b);
    g[3] = R(0.5) * (a - b);
    g[2] = R(0.5) * (c + d);
    g[4] = R(0.5) * (c - d);
    g[5] = R(0.25) * (u1 + v1);
    g[7] = R(0.25) * (u1 - v1);
    g[6] = R(0.25) * (u2 + v2);
    g[8] = R(0.25) * (u2 - v2);
}

// Conservative Allen-Cahn cascaded collision (Sec. 5) with omega_1 = omega_2 =
// omphi and the other rates 1; the first-order equilibria carry M theta n.
//
// With every rate above first order equal to 1 the cascade leaves all central
// moments (about u) of order two and higher at their equilibria, phi/3 for the
// two second-order, phi/9 for the fourth-order and zero for the others, and
// relaxes only the two first-order central moments: a = k10' - ux phi with
// k10' = k10 + omphi (phi ux + M theta n_x - k10), and b likewise.  A D2Q9
// distribution with central moments kappa_ij is sum_ij kappa_ij B_i(e_x) B_j(e_y),
// where B_0, B_1, B_2 are the three-velocity weights of central moments (1,0,0),
// (0,1,0), (0,0,1) about u; here that sum collapses to
//   f~ = phi W(e_x) W(e_y) + a D(e_x) V(e_y) + b V(e_x) D(e_y)
// with W = B_0 + B_2/3 (mean u, central second moment 1/3), D = B_1 and V = B_0.
// This equals the cascade step for step up to rounding (about 90 operations
// instead of 160).  The rest direction is taken from the balance of phi,
// f~_0 = sum f - sum_{a>0} f~_a: the weights hold the inexact constants 1/6 and
// 2/3, and summing them would bias sum f~ by the same rounding at every node and
// step (a drift of sum phi growing linearly in time).  Shifted storage stores
// f~ - w sh; the first moments of the shift vanish, so k10 and k01 are taken from
// the stored values directly, and sum f is the sum of the stored values.
template <class R>
struct Axis3 {  // values at e = -1, 0, +1
    R m, z, p;
};
template <class R>
__device__ __forceinline__ void ace_axis(R u, Axis3<R>& W, Axis3<R>& D, Axis3<R>& V) {
    const R u2 = u * u;
    const R hw = R(0.5) * u2 + R(1.0 / 6.0), hv = R(0.5) * u2, hu = R(0.5) * u;
    W.m = hw - hu; W.z = R(2.0 / 3.0) - u2; W.p = hw + hu;
    D.m = u - R(0.5); D.z = R(-2) * u; D.p = u + R(0.5);
    V.m = hv - hu; V.z = R(1) - u2; V.p = hv + hu;
}
// From the held moments of the pulled f (m.tot is read only when shifted).
template <class R, bool SH = false>
__device__ __forceinline__ void ace_collide(R f[9], const FMom<R>& m, R phi, R ux, R uy, R Mth_x, R Mth_y,
                                            R omphi, R sh = R(0)) {
    const R tot = SH ? m.tot : phi;  // sum of the stored values
    const R k10 = m.k10, k01 = m.k01;
    const R a = k10 + omphi * (phi * ux + Mth_x - k10) - ux * phi;
    const R b = k01 + omphi * (phi * uy + Mth_y - k01) - uy * phi;
    Axis3<R> Wx, Dx, Vx, Wy, Dy, Vy;
    ace_axis(ux, Wx, Dx, Vx);
    ace_axis(uy, Wy, Dy, Vy);
    const Axis3<R> P{phi * Wx.m, phi * Wx.z, phi * Wx.p};
    const Axis3<R> A{a * Dx.m, a * Dx.z, a * Dx.p};
    const Axis3<R> B{b * Dy.m, b * Dy.z, b * Dy.p};
    // direction (i, j) -> P_i W_j + A_i V_j + Vx_i B_j, less w sh when shifted
    const R s1 = SH ? sh * R(1.0 / 9.0) : R(0), s5 = SH ? sh * R(1.0 / 36.0) : R(0);
    f[1] = P.p * Wy.z - s1 + A.p * Vy.z + Vx.p * B.z;
    f[2] = P.z * Wy.p - s1 + A.z * Vy.p + Vx.z * B.p;
    f[3] = P.m * Wy.z - s1 + A.m * Vy.z + Vx.m * B.z;
    f[4] = P.z * Wy.m - s1 + A.z * Vy.m + Vx.z * B.m;
    f[5] = P.p * Wy.p - s5 + A.p * Vy.p + Vx.p * B.p;
    f[6] = P.m * Wy.p - s5 + A.m * Vy.p + Vx.m * B.p;
    f[7] = P.m * Wy.m - s5 + A.m * Vy.m + Vx.m * B.m;
    f[8] = P.p * Wy.m - s5 + A.p * Vy.m + Vx.p * B.m;
    f[0] = tot - (((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8])));
}
// From the nine pulled values, collided in place.
template <class R, bool SH = false>
__device__ __forceinline__ void ace_collide(R f[9], R phi, R ux, R uy, R Mth_x, R Mth_y, R omphi,
                                            R sh = R(0)) {
    FMom<R> m;
    hold(m, f);
    ace_collide<R, SH>(f, m, phi, ux, uy, Mth_x, Mth_y, omphi, sh);
}

// --------------------------------------------------- SRT collisions (Sec. 7)

// Single-relaxation-time comparison models: BGK relaxation at one rate toward the
// second-order Hermite equilibrium with the cascaded scheme's zeroth to second
// moments, plus the Hermite-2 form of the same source moments times (1 - om/2).
// With c^2 = 1/3 the expansion of a distribution with moments (a0, a1, A2) is
// w_a [a0 + 3 e.a1 + 4.5 (A2 - a0/3 I):(e e) - 1.5 tr(A2 - a0/3 I)].

// Hydrodynamic: equilibrium w_a [p + rho (e.u) + rho (1.5 (e.u)^2 - 0.5 u^2)];
// source w_a [F_p.u + e.F_t + 4.5 A:(e e) - 1.5 tr A] with A the second-order
// source moments less c^2 F_p.u I.  Rate omv = omega(nu(phi)).
template <class R, bool SH = false>
__device__ __forceinline__ void hydro_srt(R g[9], const NodeOut<R>& o, R sh = R(0)) {
    const R ux = o.ux, uy = o.uy, om = o.omv, hw = R(1) - R(0.5) * om;
    const R Sx = o.Ftx + o.Fpx, Sy = o.Fty + o.Fpy;
    const R Axx = R(2.0 / 3.0) * Sx * ux, Ayy = R(2.0 / 3.0) * Sy * uy;
    const R Axy = R(1.0 / 3.0) * (Sx * uy + Sy * ux);
    const R peq = o.p - R(0.5) * o.rho * (ux * ux + uy * uy);
    const R s0 = (o.Fpx * ux + o.Fpy * uy) - R(1.5) * (Axx + Ayy);
    auto upd = [&](int a, R w, int ex, int ey) {
        const R eu = R(ex) * ux + R(ey) * uy;
        const R eF = R(ex) * o.Ftx + R(ey) * o.Fty;
        const R AE = R(ex * ex) * Axx + R(ey * ey) * Ayy + R(2 * ex * ey) * Axy;
        const R geq = w * (peq + o.rho * (eu + R(1.5) * eu * eu));
        const R src = w * (s0 + eF + R(4.5) * AE);
        const R ga = SH ? g[a] + w * sh : g[a];  // unshifted value
        g[a] += om * (geq - ga) + hw * src;
    };
    const R w0 = R(4.0 / 9.0), w1 = R(1.0 / 9.0), w5 = R(1.0 / 36.0);
    upd(0, w0, 0, 0);
    upd(1, w1, 1, 0); upd(2, w1, 0, 1); upd(3, w1, -1, 0); upd(4, w1, 0, -1);
    upd(5, w5, 1, 1); upd(6, w5, -1, 1); upd(7, w5, -1, -1); upd(8, w5, 1, -1);
}

// Conservative Allen-Cahn: equilibrium w_a [phi (1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u^2)
// + 3 e.(M theta n)], every moment at rate omphi.
template <class R, bool SH = false>
__device__ __forceinline__ void ace_srt(R f[9], R phi, R ux, R uy, R Mth_x, R Mth_y, R om,
                                        R sh = R(0)) {
    const R tot = SH ? sum9(f) : phi;  // sum of the stored values
    const R base = phi * (R(1) - R(1.5) * (ux * ux + uy * uy));
    auto upd = [&](int a, R w, int ex, int ey) {
        const R eu = R(ex) * ux + R(ey) * uy;
        const R en = R(ex) * Mth_x + R(ey) * Mth_y;
        const R feq = w * (base + phi * (R(3) * eu + R(4.5) * eu * eu) + R(3) * en);
        const R fa = SH ? f[a] + w * sh : f[a];  // unshifted value
        f[a] += om * (feq - fa);
    };
    const R w1 = R(1.0 / 9.0), w5 = R(1.0 / 36.0);
    upd(1, w1, 1, 0); upd(2, w1, 0, 1); upd(3, w1, -1, 0); upd(4, w1, 0, -1);
    upd(5, w5, 1, 1); upd(6, w5, -1, 1); upd(7, w5, -1, -1); upd(8, w5, 1, -1);
    // rest direction from the balance of phi (the rounded weights would bias sum f)
    f[0] = tot - (((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8])));
}

// ------------------------------------------------------------- fused kernel

// What the collisions read of the rows pulled for phi (two rows ahead of the
// collision) and for pbar (one row ahead) stays in registers until their row
// collides: three moments of f and four of gbar for the cascaded pair, the nine
// values for the SRT pair.  PF_PREFETCH: each row iteration starts by issuing the
// pulls of the next one (f at the next leading row, gbar at the next pbar row)
// into registers of the stored type; they are converted and reduced to the held
// moments when the iteration ends, so those loads are in flight through the
// barriers, the stencils and both collisions (18 values more per lane).
//
// Register budget (resident waves per SIMD the kernels are built for): holding
// moments, the cascaded kernels without prefetching need about 110 VGPRs in FP64
// (four waves) and 85-95 in FP32 and 16-bit storage (five, so that two workgroups
// of nine waves fit a CU); the FP64 prefetching and SRT kernels about 145-165
// (three, which is also what a 9-wave 516-lane workgroup gets on one SIMD); the
// rest fits in ST::waves.
template <class ST, int PF, int COLL>
constexpr int fused_waves() {
    const bool lean = PF == PF_HOLD && COLL != COLL_SRT;
    if (ST::waves == 2) return lean ? 4 : 3;
    return lean ? 5 : ST::waves;
}

//
// WALLS false: the lattices of the launch have no walls (periodic in x and y).
// The wall kinds are then compile-time zero and the source selection of every
// pull reduces to the periodic rows; this removes about 45% of the loop's scalar
// and 5-15% of its vector instructions, which the 16-bit kernels feel (+12%).
template <int N>
using IC = std::integral_constant<int, N>;

// Whether a TX-lane workgroup's strip of TX - 4 columns is whole 128-byte lines.
template <class ST, int TX>
constexpr bool kStripLines = ((TX - 4) * (int)sizeof(typename ST::T)) % 128 == 0;

//
// NT: nontemporal stores, for launches in which every stored row segment is whole
// cache lines (strips of a multiple of 128 bytes, kStripLines, and rows of one as
// well, LatDesc::ntstore): on the 8192^2 grid they run FP64 2%, FP32 5% and fp16
// 4% faster.  Partial lines (narrow or odd-width lattices, 252- and 508-column
// strips) merge in L2 instead; streamed, they cost the uneven batch 7%.
template <class ST, int TX, int MODE, int PF, int COLL = COLL_CASCADED, bool WALLS = true, bool NT = false>
__global__ void __launch_bounds__(TX) __attribute__((amdgpu_waves_per_eu(fused_waves<ST, PF, COLL>())))
lb_fused(const LatDesc* __restrict__ descs, const WorkItem* __restrict__ items, int n_items, int parity) {
    using R = typename ST::R;
    using T = typename ST::T;
    // Role-based register pipeline (see below): the coupled cascaded step with 16-
    // or 32-bit storage without walls.  Elsewhere it is not used: in FP64 it
    // spills (168 VGPRs with prefetching), so would the SRT kernels, and the wall logic unrolled six times
    // (about 6000 instructions) outgrows the instruction cache (a batch with walled
    // lattices ran 14% slower with it).
    constexpr bool kRoles = MODE == MODE_STEP && COLL == COLL_CASCADED && sizeof(T) < 8 && !WALLS;
    constexpr int RING = kRoles ? 6 : 4;  // rows held in each LDS ring
    __shared__ R s_phi[RING][TX];
    __shared__ R s_pb[RING][TX];
    __shared__ R s_na[RING][TX];  // n_x (geometric) or mu_phi (chemical potential)
    __shared__ R s_nb[RING][TX];  // n_y (geometric)
    const int t = lane_slot<TX>(threadIdx.x);  // column slot of this lane

    for (int wi = blockIdx.x; wi < n_items; wi += gridDim.x) {
        const WorkItem it = items[wi];
        if (it.y1 <= it.y0) continue;  // padding item (uniform over the block)
        const LatDesc& D = descs[it.inst];
        const int nx = D.nx, ny = D.ny, chem = D.st_form;
        const int wall = WALLS ? D.wall_y : WALL_NONE, wallx = WALLS ? D.wall_x : WALL_NONE;
        const KConst<R> K = load_const<R>(D);
        // Stochastic rounding of 16-bit stores: the step count of the state read now
        // seeds the random bits, and the launch records the count of the state it
        // writes (every work item of the lattice stores the same value).
        uint32_t tseed = 0;
        bool sr = false;
        if constexpr (ST::shifted && MODE == MODE_STEP) {
            sr = D.sround != 0;
            if (sr) {
                const uint32_t tv = D.tstep[parity];
                if (threadIdx.x == 0) D.tstep[parity ^ 1] = tv + 1u;
                tseed = seed_step(tv);
            }
        }
        const double* ktab = D.surf ? D.ktab : nullptr;  // per-row Langmuir table
        const T* __restrict__ src = reinterpret_cast<const T*>(D.buf[parity]);
        T* __restrict__ dst = reinterpret_cast<T*>(D.buf[parity ^ 1]);
        const T* __restrict__ srcg = src + 9 * nx;  // gbar values of row 0
        const int w = min(TX - 4, nx - it.x0);  // interior columns of this strip
        const bool inA = t < w + 4;              // phi cells
        const bool inB = t >= 1 && t < w + 3;    // pbar and normal cells
        const bool inF = t >= 2 && t < w + 2;    // collided cells
        // this lane's column: halo lanes wrap, or mirror across x walls (ghost
        // values); lanes past the strip are idle and park on column 0
        int xc = inA ? map_row(it.x0 - 2 + t, nx, wallx) : 0;
        int xm = xc == 0 ? nx - 1 : xc - 1;
        int xp = xc == nx - 1 ? 0 : xc + 1;

        // Register pipeline: the f pulled at the leading row is collided two
        // iterations later, the gbar one iteration later, and the gradient and
        // normal found for row L - 1 serve its collision in the next iteration.
        // By copies: F[0], G[0] and entry 0 take the new values, and each
        // iteration ends by shifting F[0] -> F[1] -> F[2], G[0] -> G[1] and entry
        // 0 -> 1.  By roles (kRoles): the values stay where they were written,
        // in F[k % 3], G[k % 2] and entry k % 2, the rings hold the row leading in
        // iteration k in slot k % 6, and the loop is unrolled six times so that
        // every role and slot is a constant: nothing is moved between iterations.
        // The prefetched rows (PF_PREFETCH) are then reduced into the entries the
        // collision has just consumed, F[(k + 1) % 3] and G[(k + 1) % 2], which are
        // the next iteration's leading ones.
        // Each F and G entry holds what the collision reads of its row (FMom,
        // GMom), or the nine values for the SRT collisions.
        constexpr bool kMom = COLL != COLL_SRT;
        using HF = std::conditional_t<kMom, FMom<R>, Vals9<R>>;
        using HG = std::conditional_t<kMom, GMom<R>, Vals9<R>>;
        HF F[3];
        HG G[2];
        T nf[9], ng[9];  // next rows' pulls in flight (PF_PREFETCH)
        R Pn = R(0);     // sum of the prefetched gbar (PF_PREFETCH)
        R Dx[2], Dy[2], Dm[2], Nx[2], Ny[2];  // grad phi, |grad phi|^2, normal
        {
            R z[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                z[a] = R(0);
                nf[a] = ng[a] = T(0);
            }
            hold(F[0], z);
            F[2] = F[1] = F[0];
            hold(G[0], z);
            G[1] = G[0];
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) Dx[j] = Dy[j] = Dm[j] = Nx[j] = Ny[j] = R(0);

        const int H = it.y1 - it.y0;
        constexpr bool ahead = PF == PF_PREFETCH && MODE == MODE_STEP;
        // One row iteration.  S0..S3: ring slots of rows L, L - 1, L - 2, L - 3;
        // fo, ft: F entries of the f pulled now and two iterations ago; go, gt: G
        // entries of the gbar pulled now and one iteration ago; dw, dr: entries of
        // the gradient found now and one iteration ago.
        auto row_step = [&](const int k, auto S0, auto S1, auto S2, auto S3, auto fo, auto ft, auto go, auto gt,
                            auto dw, auto dr) __attribute__((always_inline)) {
            HF& f0 = F[fo];
            const HF& f2 = F[ft];
            HG& g0 = G[go];
            const HG& g1 = G[gt];
            const int L = it.y0 - 2 + k;
            if constexpr (!kBufIO<ST>) lane_columns_in_loop(xc, xm, xp);
            if (ahead && k + 1 < H + 4) {  // the next iteration's pulls
                if (inA) pull9<ST, kBufIO<ST>, true>(src, nx, ny, wall, wallx, xc, xm, xp, map_row(L + 1, ny, wall), nf);
                if (k >= 2 && inB) pull9<ST, kBufIO<ST>, true>(srcg, nx, ny, wall, wallx, xc, xm, xp, map_row(L, ny, wall), ng);
            }
            // ---- A: phi at the leading row
            if (inA) {
                if (!ahead || k == 0) {
                    R v[9];
                    pull9<ST, kBufIO<ST>>(src, nx, ny, wall, wallx, xc, xm, xp, map_row(L, ny, wall), v);
                    hold(f0, v);
                }
                R ph = held_sum(f0);
                if constexpr (ST::shifted) ph += K.shf;
                s_phi[S0][t] = ph;
            }
            // ---- B: pbar one row behind
            if (k >= 2 && inB) {
                const int Lg = L - 1;
                R pb = Pn;
                if (!ahead || k == 2) {
                    R v[9];
                    pull9<ST, kBufIO<ST>>(srcg, nx, ny, wall, wallx, xc, xm, xp, map_row(Lg, ny, wall), v);
                    hold(g0, v);
                    pb = sum9(v);
                }
                if constexpr (ST::shifted) pb += K.shg;
                s_pb[S1][t] = pb;
            }
            __syncthreads();
            // ---- D: gradient, normal or chemical potential at row L-1
            if (k >= 2 && inB) {
                const int Ln = L - 1;
                const R* rs = s_phi[S2];
                const R* rm = s_phi[S1];
                const R* rn = s_phi[S0];
                R gx, gy;
                grad3x3(rs, rm, rn, t, gx, gy);
                const R m2 = gx * gx + gy * gy;
                R ix, iy;
                unit_normal(gx, gy, m2, ix, iy);
                if (chem) {
                    const R yrow = R(map_row(Ln, ny, wall));
                    const R ph = rm[t];
                    const R beta = K.be_a + K.be_b * yrow;
                    const R kap = K.ka_a + K.ka_b * yrow;
                    s_na[S1][t] = R(4) * beta * (ph - R(1)) * ph * (ph - R(0.5)) -
                                      kap * lap3x3(rs, rm, rn, t);
                } else {
                    s_na[S1][t] = ix;
                    s_nb[S1][t] = iy;
                }
                Dx[dw] = gx; Dy[dw] = gy; Dm[dw] = m2; Nx[dw] = ix; Ny[dw] = iy;
            }
            __syncthreads();
            // ---- F: collide row C = L - 2
            if (k >= 4) {
                const int C = L - 2;
                NodeIn<R> in;
                NodeOut<R> o;
                uint32_t idx = 0;
                if (inF) {
                    in.phi = s_phi[S2][t];
                    in.pbar = s_pb[S2][t];
                    in.dphx = Dx[dr]; in.dphy = Dy[dr]; in.m2 = Dm[dr]; in.nx = Nx[dr]; in.ny = Ny[dr];
                    row_kappa(K, ktab, ny, C, in.kt, in.dkt);
                    in.divn = R(0); in.dmux = R(0); in.dmuy = R(0);
                    grad3x3(s_pb[S3], s_pb[S2], s_pb[S1], t, in.dpx, in.dpy);
                    if (chem) {
                        grad3x3(s_na[S3], s_na[S2], s_na[S1], t, in.dmux, in.dmuy);
                    } else {
                        R a1, a2, b1, b2;
                        grad3x3(s_na[S3], s_na[S2], s_na[S1], t, a1, a2);
                        grad3x3(s_nb[S3], s_nb[S2], s_nb[S1], t, b1, b2);
                        in.divn = a1 + b2;
                    }
                    R jx, jy;
                    held_first(g1, jx, jy);
                    o = node_macro<R>(K, chem, in, jx, jy);
                    idx = (uint32_t)C * (uint32_t)nx + (uint32_t)xc;
                }
                if constexpr (MODE == MODE_STEP) {
                    // gbar first: fewer values stay live across the second collision
                    const uint32_t hn = ST::shifted && sr ? node_hash(tseed, xc, C) : 0u;
                    if (inF) {
                        R v[9];
                        if constexpr (COLL == COLL_SRT) {
                            for (int a = 0; a < 9; ++a) v[a] = g1.v[a];
                            hydro_srt<R, ST::shifted>(v, o, K.shg);
                        } else {
                            hydro_collide<R, ST::shifted, COLL != COLL_PRINTED>(v, o, g1.nd, g1.xd, K.shg);
                        }
                        store_collided<ST, kBufIO<ST>, NT>(sr, row_at(dst, C, nx), nx, 9, xc, v, hn);
                    }
                    if (inF) {
                        const R Mth = K.M * (K.four_W * in.phi * (R(1) - in.phi));
                        R v[9];
                        if constexpr (COLL == COLL_SRT) {
                            for (int a = 0; a < 9; ++a) v[a] = f2.v[a];
                            ace_srt<R, ST::shifted>(v, in.phi, o.ux, o.uy, Mth * in.nx, Mth * in.ny, K.omphi, K.shf);
                        } else {
                            ace_collide<R, ST::shifted>(v, f2, in.phi, o.ux, o.uy, Mth * in.nx, Mth * in.ny, K.omphi,
                                                        K.shf);
                        }
                        store_collided<ST, kBufIO<ST>, NT>(sr, row_at(dst, C, nx), nx, 0, xc, v, hn);
                    }
                } else if constexpr (MODE == MODE_FIELDS) {
                    if (inF) {
                        double* F = D.fields;
                        const int64_t N = (int64_t)nx * ny;
                        F[idx] = (double)in.phi;
                        F[N + idx] = (double)o.p;
                        F[2 * N + idx] = (double)o.ux;
                        F[3 * N + idx] = (double)o.uy;
                    }
                } else {
                    if (inF) {
                        double* F = D.fields;
                        const int64_t N = (int64_t)nx * ny;
                        F[idx] = (double)in.dphx;
                        F[N + idx] = (double)in.dphy;
                        F[2 * N + idx] = (double)in.nx;
                        F[3 * N + idx] = (double)in.ny;
                        F[4 * N + idx] = (double)in.divn;
                        F[5 * N + idx] = (double)o.Ftx;
                        F[6 * N + idx] = (double)o.Fty;
                        F[7 * N + idx] = (double)o.Fpx;
                        F[8 * N + idx] = (double)o.Fpy;
                    }
                }
            }
        };
        // The prefetched rows, converted and reduced into F entry fn and G entry gn.
        auto take_prefetch = [&](HF& fn, HG& gn) __attribute__((always_inline)) {
            R v[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) v[a] = ST::ld(nf[a]);
            hold(fn, v);
#pragma unroll
            for (int a = 0; a < 9; ++a) v[a] = ST::ld(ng[a]);
            hold(gn, v);
            Pn = sum9(v);
        };
        if constexpr (kRoles) {
            // slots and roles of iteration k = k0 + PH
            auto phase = [&](auto Pc, const int k) __attribute__((always_inline)) {
                constexpr int PH = decltype(Pc)::value;
                row_step(k, IC<PH>{}, IC<(PH + 5) % 6>{}, IC<(PH + 4) % 6>{}, IC<(PH + 3) % 6>{}, IC<PH % 3>{},
                         IC<(PH + 1) % 3>{}, IC<PH % 2>{}, IC<(PH + 1) % 2>{}, IC<PH % 2>{}, IC<(PH + 1) % 2>{});
                if constexpr (ahead) take_prefetch(F[(PH + 1) % 3], G[(PH + 1) % 2]);
            };
            for (int k0 = 0; k0 < H + 4; k0 += 6) {
                phase(IC<0>{}, k0);
                if (k0 + 1 < H + 4) phase(IC<1>{}, k0 + 1);
                if (k0 + 2 < H + 4) phase(IC<2>{}, k0 + 2);
                if (k0 + 3 < H + 4) phase(IC<3>{}, k0 + 3);
                if (k0 + 4 < H + 4) phase(IC<4>{}, k0 + 4);
                if (k0 + 5 < H + 4) phase(IC<5>{}, k0 + 5);
            }
        } else {
            for (int k = 0; k < H + 4; ++k) {
                const int L = it.y0 - 2 + k;
                row_step(k, L & 3, (L - 1) & 3, (L - 2) & 3, (L - 3) & 3, IC<0>{}, IC<2>{}, IC<0>{}, IC<1>{}, IC<0>{},
                         IC<1>{});
                // ---- shift the register pipeline
                F[2] = F[1];
                F[1] = F[0];
                G[1] = G[0];
                if constexpr (ahead) take_prefetch(F[0], G[0]);
                Dx[1] = Dx[0]; Dy[1] = Dy[0]; Dm[1] = Dm[0]; Nx[1] = Nx[0]; Ny[1] = Ny[0];
            }
        }
        __syncthreads();  // the rings are reused by the next work item
    }
}

// ------------------------------------------------- phase field only (Sec. 6.1)

// The conservative Allen-Cahn step alone under an imposed velocity (planes ux, uy
// of the compute type at D.vel, stride D.plane).  Same work items and lane layout
// as lb_fused (slot t at column x0 - 2 + t, strips of TX - 4 columns); the
// pipeline lags one row: pull f at row L into the phi ring, then take grad phi,
// n and theta at row L - 1 and collide it.  One barrier per row suffices with a
// ring of four rows.  COLL selects the cascaded or the SRT collision.  Of the
// pulled row the cascaded collision keeps the sum and the first moments (FMom),
// the SRT one the nine values.  kPF (32- and 64-bit storage): each iteration
// issues the next row's pull (stored type, in registers) and the velocity of the
// row it collides next as soon as the current ones are read, so the loads fly
// through the barrier, the stencil and the collision: FP32 +5%, FP64 with the
// SRT collision +5% on the 8192^2 grid, FP64 with the cascaded one unchanged;
// the 16-bit kernels ran 14% slower with it and pull each row where they use it.
template <class ST, int TX, int MODE, int COLL, bool WALLS = true>
__global__ void __launch_bounds__(TX) lb_ace(const LatDesc* __restrict__ descs,
                                             const WorkItem* __restrict__ items, int n_items,
                                             int parity) {
    using R = typename ST::R;
    using T = typename ST::T;
    constexpr bool kMom = COLL != COLL_SRT;
    using HF = std::conditional_t<kMom, FMom<R>, Vals9<R>>;
    constexpr bool kPF = sizeof(T) >= 4;
    __shared__ R s_phi[4][TX];
    const int t = lane_slot<TX>(threadIdx.x);  // column slot of this lane

    for (int wi = blockIdx.x; wi < n_items; wi += gridDim.x) {
        const WorkItem it = items[wi];
        if (it.y1 <= it.y0) continue;
        const LatDesc& D = descs[it.inst];
        const int nx = D.nx, ny = D.ny;
        const int wall = WALLS ? D.wall_y : WALL_NONE, wallx = WALLS ? D.wall_x : WALL_NONE;
        const int64_t P = D.plane;  // stride of the two velocity planes
        const R shf = R(D.shift_f), four_W = R(D.four_W), Mm = R(D.M), omphi = R(D.omphi);
        const T* __restrict__ src = reinterpret_cast<const T*>(D.buf[parity]);
        T* __restrict__ dst = reinterpret_cast<T*>(D.buf[parity ^ 1]);
        const R* __restrict__ vel = reinterpret_cast<const R*>(D.vel);
        uint32_t tseed = 0;  // stochastic rounding of 16-bit stores, as in lb_fused
        bool sr = false;
        if constexpr (ST::shifted && MODE == MODE_STEP) {
            sr = D.sround != 0;
            if (sr) {
                const uint32_t tv = D.tstep[parity];
                if (threadIdx.x == 0) D.tstep[parity ^ 1] = tv + 1u;
                tseed = seed_step(tv);
            }
        }
        const int w = min(TX - 4, nx - it.x0);
        const bool inA = t < w + 4;
        const bool inF = t >= 2 && t < w + 2;
        int xc = inA ? map_row(it.x0 - 2 + t, nx, wallx) : 0;
        int xm = xc == 0 ? nx - 1 : xc - 1;
        int xp = xc == nx - 1 ? 0 : xc + 1;

        const int H = it.y1 - it.y0;
        HF f1{};       // what the collision reads of the pulled row one behind
        T nf[9];       // the next row's pull in flight (kPF)
        R nux = R(0), nuy = R(0);  // velocity of the row collided next (kPF)
        if constexpr (kPF)
            if (inA)
                pull9<ST, kBufIOAce<ST>, true>(src, nx, ny, wall, wallx, xc, xm, xp, map_row(it.y0 - 1, ny, wall), nf);
        for (int k = 0; k < H + 2; ++k) {
            const int L = it.y0 - 1 + k;
            if constexpr (!kBufIOAce<ST>) lane_columns_in_loop(xc, xm, xp);
            HF f0{};
            R ux = nux, uy = nuy;  // row L - 1
            if (inA) {
                R v[9];
                if constexpr (kPF) {
#pragma unroll
                    for (int a = 0; a < 9; ++a) v[a] = ST::ld(nf[a]);
                    if (k + 1 < H + 2)
                        pull9<ST, kBufIOAce<ST>, true>(src, nx, ny, wall, wallx, xc, xm, xp,
                                                       map_row(L + 1, ny, wall), nf);
                    if (inF && k >= 1 && k <= H) {
                        const uint32_t idx = (uint32_t)L * (uint32_t)nx + (uint32_t)xc;
                        nux = vel[idx];
                        nuy = vel[P + idx];
                    }
                } else {
                    pull9<ST, kBufIOAce<ST>>(src, nx, ny, wall, wallx, xc, xm, xp, map_row(L, ny, wall), v);
                }
                hold(f0, v);
                R ph = held_sum(f0);
                if constexpr (ST::shifted) ph += shf;
                s_phi[L & 3][t] = ph;
            }
            __syncthreads();
            if (k >= 2 && inF) {
                const int C = L - 1;
                const R phi = s_phi[C & 3][t];
                R gx, gy, ix, iy;
                grad3x3(s_phi[(C - 1) & 3], s_phi[C & 3], s_phi[(C + 1) & 3], t, gx, gy);
                const R m2 = gx * gx + gy * gy;
                unit_normal(gx, gy, m2, ix, iy);
                const uint32_t idx = (uint32_t)C * (uint32_t)nx + (uint32_t)xc;
                if constexpr (!kPF) {
                    ux = vel[idx];
                    uy = vel[P + idx];
                }
                if constexpr (MODE == MODE_STEP) {
                    const R Mth = Mm * (four_W * phi * (R(1) - phi));
                    R f[9];
                    if constexpr (COLL == COLL_SRT) {
#pragma unroll
                        for (int a = 0; a < 9; ++a) f[a] = f1.v[a];
                        ace_srt<R, ST::shifted>(f, phi, ux, uy, Mth * ix, Mth * iy, omphi, shf);
                    } else {
                        ace_collide<R, ST::shifted>(f, f1, phi, ux, uy, Mth * ix, Mth * iy, omphi, shf);
                    }
                    store_collided<ST, kBufIOAce<ST>, false>(sr, row_at(dst, C, nx), nx, 0, xc, f,
                                                       ST::shifted && sr ? node_hash(tseed, xc, C) : 0u);
                } else {
                    double* F = D.fields;
                    const int64_t N = (int64_t)nx * ny;
                    if constexpr (MODE == MODE_FIELDS) {
                        F[idx] = (double)phi;
                        F[N + idx] = 0.0;
                        F[2 * N + idx] = (double)ux;
                        F[3 * N + idx] = (double)uy;
                    } else {
                        F[idx] = (double)gx;
                        F[N + idx] = (double)gy;
                        F[2 * N + idx] = (double)ix;
                        F[3 * N + idx] = (double)iy;
                        for (int q = 4; q < 9; ++q) F[q * N + idx] = 0.0;
                    }
                }
            }
            f1 = f0;
        }
        __syncthreads();
    }
}

}  // namespace cmlb
