// lb_aux.hip -- kernels around the step (gfx950): state set-up and read-out,
// the built-in initial phase field, FP64 diagnostics and the copy reference.
#include "lb_internal.hpp"

namespace cmlb {

// ------------------------------------------------ state set-up and read-out

__device__ __forceinline__ int ex_of(int a) {
    return (a == 1 || a == 5 || a == 8) ? 1 : ((a == 3 || a == 6 || a == 7) ? -1 : 0);
}
__device__ __forceinline__ int ey_of(int a) {
    return (a == 2 || a == 5 || a == 6) ? 1 : ((a == 4 || a == 7 || a == 8) ? -1 : 0);
}
__device__ __forceinline__ int opp_of(int a) {
    return a == 0 ? 0 : (a <= 4 ? ((a + 1) & 3) + 1 : ((a - 3) & 3) + 5);
}
// Direction with e_y reversed (specular reflection at a wall y = const).
__device__ __forceinline__ int miry_of(int a) {
    switch (a) {
    case 2: return 4;
    case 4: return 2;
    case 5: return 8;
    case 8: return 5;
    case 6: return 7;
    case 7: return 6;
    }
    return a;
}
__device__ __forceinline__ int wrapx(int x, int nx) { return x < 0 ? x + nx : (x >= nx ? x - nx : x); }

__device__ __forceinline__ int mirx_of(int a) {
    switch (a) {
    case 1: return 3;
    case 3: return 1;
    case 5: return 6;
    case 6: return 5;
    case 7: return 8;
    case 8: return 7;
    }
    return a;
}

// Where the population arriving at node (x, y) in direction a is stored (as the
// previous step's post-collision value): direction *b at node (*xs, *ys).
// Inside: f~_a(x - e_a).  Beyond one wall: bounce-back takes the opposite
// direction at the same node; specular reflection takes the mirrored direction at
// the node the particle left along the wall.  Beyond an x and a y wall at once:
// bounce-back.  For every lattice this is a bijection of (node, direction) onto
// the stored values, so the set-up kernels below scatter through it.
__device__ __forceinline__ void pull_source(const LatDesc& D, int a, int x, int y, int* b, int* xs,
                                            int* ys) {
    const int nx = D.nx, ny = D.ny;
    const int is = x - ex_of(a), js = y - ey_of(a);
    const bool outy = D.wall_y && (js < 0 || js >= ny);
    const bool outx = D.wall_x && (is < 0 || is >= nx);
    if ((outy && outx) || (outy && D.wall_y == WALL_BOUNCE) || (outx && D.wall_x == WALL_BOUNCE)) {
        *b = opp_of(a); *xs = x; *ys = y;
    } else if (outy) {
        *b = miry_of(a); *xs = wrapx(is, nx); *ys = y;
    } else if (outx) {
        *b = mirx_of(a); *xs = x; *ys = wrapx(js, ny);
    } else {
        *b = a; *xs = wrapx(is, nx); *ys = wrapx(js, ny);
    }
}

// Element of stored value q (0..8 f, 9..17 gbar) of node (x, y): the row-interleaved
// layout of the step kernels.
__device__ __forceinline__ int64_t sidx(int nx, int q, int y, int x) {
    return ((int64_t)y * 18 + q) * nx + x;
}

// State at t = 0: every arriving population is f_a = w_a phi0, gbar_a = 0.
template <class ST>
__global__ void k_init(const LatDesc* __restrict__ dp, const double* __restrict__ phi0, int cur) {
    const LatDesc& D = *dp;
    const int nx = D.nx, ny = D.ny;
    const int64_t N = (int64_t)nx * ny;
    using T = typename ST::T;
    T* buf = reinterpret_cast<T*>(D.buf[cur]);
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < N;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(k / nx), x = (int)(k % nx);
        for (int a = 0; a < 9; ++a) {
            int b, xs, ys;
            pull_source(D, a, x, y, &b, &xs, &ys);
            const double w = wgt(a);  // w_b = w_a for opposite and mirrored directions
            buf[sidx(nx, b, ys, xs)] = ST::st((typename ST::R)(w * phi0[k] - w * D.shift_f));
            buf[sidx(nx, 9 + b, ys, xs)] = ST::st((typename ST::R)(0.0 - w * D.shift_g));
        }
    }
}

// Stores one staged post-streaming FP64 plane a of f (which = 0) or gbar
// (which = 1): the value arriving at each node goes where the next pull finds it.
template <class ST>
__global__ void k_set_plane(const LatDesc* __restrict__ dp, const double* __restrict__ stage,
                            int a, int which, int cur) {
    const LatDesc& D = *dp;
    const int nx = D.nx, ny = D.ny;
    const int64_t N = (int64_t)nx * ny;
    using T = typename ST::T;
    T* buf = reinterpret_cast<T*>(D.buf[cur]);
    const int q0 = which ? 9 : 0;
    const double sh = which ? D.shift_g : D.shift_f;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < N;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(k / nx), x = (int)(k % nx);
        int b, xs, ys;
        pull_source(D, a, x, y, &b, &xs, &ys);
        buf[sidx(nx, q0 + b, ys, xs)] = ST::st((typename ST::R)(stage[k] - wgt(a) * sh));
    }
}

// Post-streaming FP64 plane a of f (which = 0) or gbar (which = 1).
template <class ST>
__global__ void k_get_plane(const LatDesc* __restrict__ dp, double* __restrict__ out, int a,
                            int which, int cur) {
    const LatDesc& D = *dp;
    const int nx = D.nx, ny = D.ny;
    const int64_t N = (int64_t)nx * ny;
    using T = typename ST::T;
    const T* buf = reinterpret_cast<const T*>(D.buf[cur]);
    const int q0 = which ? 9 : 0;
    const double sh = which ? D.shift_g : D.shift_f;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < N;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(k / nx), x = (int)(k % nx);
        int b, xs, ys;
        pull_source(D, a, x, y, &b, &xs, &ys);
        out[k] = (double)ST::ld(buf[sidx(nx, q0 + b, ys, xs)]) + wgt(a) * sh;
    }
}

// Langmuir law per row (Eq. Langmuirisotherm): kappa~(y) = kt0 (1 + beta ln(1 - psi))
// with psi = ps_a + ps_G y, and its derivative -kt0 beta ps_G / (1 - psi).
__global__ void k_kappa_table(const LatDesc* __restrict__ dp) {
    const LatDesc& D = *dp;
    for (int y = blockIdx.x * blockDim.x + threadIdx.x; y < D.ny; y += gridDim.x * blockDim.x) {
        const double q = 1.0 - (D.ps_a + D.ps_G * (double)y);
        D.ktab[y] = D.kt0 * (1.0 + D.lbeta * log(q));
        D.ktab[D.ny + y] = -D.kt0 * D.lbeta * D.ps_G / q;
    }
}

hipError_t launch_kappa_table(const LatDesc* d, int ny, hipStream_t s) {
    int g = (ny + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_kappa_table, dim3(g), dim3(256), 0, s, d);
    return hipGetLastError();
}

// Imposed velocity: staged FP64 planes ux, uy (N each) into the compute-type planes.
template <class R>
__global__ void k_set_vel(const LatDesc* __restrict__ dp, const double* __restrict__ stage) {
    const LatDesc& D = *dp;
    const int64_t N = (int64_t)D.nx * D.ny;
    R* vel = reinterpret_cast<R*>(D.vel);
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < N;
         k += (int64_t)gridDim.x * blockDim.x) {
        vel[k] = (R)stage[k];
        vel[D.plane + k] = (R)stage[N + k];
    }
}

hipError_t launch_set_velocity(int prec, const LatDesc* d, const double* stage, int64_t N, hipStream_t s) {
    const int bs = 256;
    int64_t g = (N + bs - 1) / bs;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    if (prec == LB_FP64) hipLaunchKernelGGL((k_set_vel<double>), dim3((int)g), dim3(bs), 0, s, d, stage);
    else hipLaunchKernelGGL((k_set_vel<float>), dim3((int)g), dim3(bs), 0, s, d, stage);
    return hipGetLastError();
}

template <class ST>
static hipError_t launch_setget(int op, const LatDesc* d, double* plane, int a, int which, int cur,
                                int64_t N, hipStream_t s) {
    const int bs = 256;
    int64_t g = (N + bs - 1) / bs;
    if (g > 65536) g = 65536;
    if (op == 0) hipLaunchKernelGGL((k_init<ST>), dim3((int)g), dim3(bs), 0, s, d, plane, cur);
    else if (op == 1) hipLaunchKernelGGL((k_set_plane<ST>), dim3((int)g), dim3(bs), 0, s, d, plane, a, which, cur);
    else hipLaunchKernelGGL((k_get_plane<ST>), dim3((int)g), dim3(bs), 0, s, d, plane, a, which, cur);
    return hipGetLastError();
}

hipError_t launch_state_op(int prec, int op, const LatDesc* d, double* plane, int a, int which,
                           int cur, int64_t N, hipStream_t s) {
    switch (prec) {
    case LB_FP64: return launch_setget<StF64>(op, d, plane, a, which, cur, N, s);
    case LB_FP32: return launch_setget<StF32>(op, d, plane, a, which, cur, N, s);
    case LB_FP32_F16: return launch_setget<StF16>(op, d, plane, a, which, cur, N, s);
    case LB_FP32_BF16: return launch_setget<StBF16>(op, d, plane, a, which, cur, N, s);
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------- built-in initial field

struct InitGeom {
    int kind, nx, ny;
    double W;
    double par[8];
};

// phi0 = 1/2 + 1/2 tanh(2 d / W) of the signed distance d of the built-in shapes
// (see LB_INIT_* in cmlb.h), one node per thread, FP64.
__global__ void k_phi_builtin(double* __restrict__ out, InitGeom g) {
    const int64_t N = (int64_t)g.nx * g.ny;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < N;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(k / g.nx), x = (int)(k % g.nx);
        double X = x, Y = y, d;
        if (g.kind == LB_INIT_DROPLET || g.kind == LB_INIT_ELLIPSE) {
            if (g.par[4] > 0) X = fmod(X, g.par[4]);
            if (g.par[5] > 0) Y = fmod(Y, g.par[5]);
            X -= g.par[0];
            Y -= g.par[1];
            const double r = hypot(X, Y);
            if (g.kind == LB_INIT_DROPLET) {
                d = g.par[3] * (g.par[2] - r);
            } else {
                const double q = sqrt((X / g.par[2]) * (X / g.par[2]) + (Y / g.par[3]) * (Y / g.par[3]));
                d = q > 0 ? r * (1.0 / q - 1.0) : fmax(g.par[2], g.par[3]);
            }
        } else {
            d = Y - g.par[0] - g.par[1] * cos(2.0 * 3.14159265358979323846 * g.par[2] * X / g.nx);
        }
        out[k] = 0.5 + 0.5 * tanh(2.0 * d / g.W);
    }
}

hipError_t launch_phi_builtin(double* out, const lb_config* c, hipStream_t s) {
    InitGeom g;
    g.kind = c->init_kind;
    g.nx = c->nx;
    g.ny = c->ny;
    g.W = c->W;
    for (int i = 0; i < 8; ++i) g.par[i] = c->init_par[i];
    const int64_t N = (int64_t)c->nx * c->ny;
    int64_t blocks = (N + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_phi_builtin, dim3((unsigned)blocks), dim3(256), 0, s, out, g);
    return hipGetLastError();
}

// ------------------------------------------------------------ diagnostics

// One block per row: partial sums over x of phi, rho, y phi, max |u|, NaN count
// (fixed tree order, so results do not depend on anything but the row).
__global__ void __launch_bounds__(256) k_diag_rows(const LatDesc* __restrict__ dp,
                                                   const double* __restrict__ F,
                                                   double* __restrict__ part) {
    const LatDesc& D = *dp;
    const int nx = D.nx, ny = D.ny;
    const int64_t N = (int64_t)nx * ny;
    const int y = blockIdx.x;
    __shared__ double s_phi[256], s_rho[256], s_max[256], s_nan[256];
    double sp = 0, sr = 0, mx = 0, nn = 0;
    for (int x = threadIdx.x; x < nx; x += 256) {
        const int64_t k = (int64_t)y * nx + x;
        const double ph = F[k], p = F[N + k], ux = F[2 * N + k], uy = F[3 * N + k];
        sp += ph;
        sr += D.rhoB + ph * D.dRho;
        const double um = sqrt(ux * ux + uy * uy);
        if (!(um <= mx) && !isnan(mx)) mx = um;  // a NaN, once met, is kept
        if (!isfinite(ph) || !isfinite(p) || !isfinite(um)) nn += 1;
    }
    s_phi[threadIdx.x] = sp; s_rho[threadIdx.x] = sr; s_max[threadIdx.x] = mx; s_nan[threadIdx.x] = nn;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            s_phi[threadIdx.x] += s_phi[threadIdx.x + st];
            s_rho[threadIdx.x] += s_rho[threadIdx.x + st];
            const double o = s_max[threadIdx.x + st];
            if (!(o <= s_max[threadIdx.x]) && !isnan(s_max[threadIdx.x])) s_max[threadIdx.x] = o;
            s_nan[threadIdx.x] += s_nan[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[4 * (int64_t)y + 0] = s_phi[0];
        part[4 * (int64_t)y + 1] = s_rho[0];
        part[4 * (int64_t)y + 2] = s_max[0];
        part[4 * (int64_t)y + 3] = s_nan[0];
    }
}

// Linear interpolation of the phi = 1/2 crossing between rows j and j + 1 of column x.
__device__ double crossing_at(const double* phi, int nx, int x, int j) {
    const double a = phi[(int64_t)j * nx + x] - 0.5, b = phi[(int64_t)(j + 1) * nx + x] - 0.5;
    return j + a / (a - b);
}
__device__ bool crosses(const double* phi, int nx, int x, int j) {
    const double a = phi[(int64_t)j * nx + x] - 0.5, b = phi[(int64_t)(j + 1) * nx + x] - 0.5;
    return (a < 0) != (b < 0);
}

// Final pass, one workgroup of 256 threads.  Thread t sums the partials of rows
// t, t + 256, ... in order and the 256 sums are then added in a fixed tree, so the
// result is the same on every run.  The tips are the first phi = 1/2 crossing from
// the bottom in column nx / 2 and the first from the top in column 0: each thread
// checks its rows, and a min / max reduction picks the crossing row.
__global__ void __launch_bounds__(256) k_diag_final(const LatDesc* __restrict__ dp, const double* __restrict__ F,
                                                    const double* __restrict__ part, double* __restrict__ out,
                                                    double step, double u_max) {
    const LatDesc& D = *dp;
    const int nx = D.nx, ny = D.ny;
    const int64_t N = (int64_t)nx * ny;
    const int t = threadIdx.x;
    __shared__ double s_sp[256], s_sr[256], s_sy[256], s_mx[256], s_nn[256];
    __shared__ int s_lo[256], s_hi[256];
    double sp = 0, sr = 0, sy = 0, mx = 0, nn = 0;
    int lo = INT_MAX, hi = -1;
    for (int y = t; y < ny; y += 256) {
        const double ph = part[4 * (int64_t)y];
        sp += ph;
        sr += part[4 * (int64_t)y + 1];
        sy += (double)y * ph;
        const double o = part[4 * (int64_t)y + 2];
        if (!(o <= mx) && !isnan(mx)) mx = o;
        nn += part[4 * (int64_t)y + 3];
    }
    for (int j = t; j + 1 < ny; j += 256) {
        if (lo == INT_MAX && crosses(F, nx, nx / 2, j)) lo = j;
        if (crosses(F, nx, 0, j)) hi = j;
    }
    s_sp[t] = sp; s_sr[t] = sr; s_sy[t] = sy; s_mx[t] = mx; s_nn[t] = nn; s_lo[t] = lo; s_hi[t] = hi;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st) {
            s_sp[t] += s_sp[t + st];
            s_sr[t] += s_sr[t + st];
            s_sy[t] += s_sy[t + st];
            const double o = s_mx[t + st];
            if (!(o <= s_mx[t]) && !isnan(s_mx[t])) s_mx[t] = o;
            s_nn[t] += s_nn[t + st];
            s_lo[t] = min(s_lo[t], s_lo[t + st]);
            s_hi[t] = max(s_hi[t], s_hi[t + st]);
        }
        __syncthreads();
    }
    if (t == 0) {
        const double nan = __longlong_as_double(0x7ff8000000000000LL);
        out[0] = step;
        out[1] = s_sp[0];
        out[2] = s_sr[0];
        out[3] = s_mx[0];
        out[4] = F[N + (int64_t)(ny / 2) * nx + nx / 2] - F[N];
        out[5] = sqrt(s_sp[0] / 3.14159265358979323846);
        out[6] = s_lo[0] == INT_MAX ? nan : crossing_at(F, nx, nx / 2, s_lo[0]);
        out[7] = s_hi[0] < 0 ? nan : crossing_at(F, nx, 0, s_hi[0]);
        out[8] = s_sy[0] / s_sp[0];
        out[9] = s_nn[0] > 0 ? 1.0 : 0.0;
        out[10] = (s_nn[0] > 0 || !(s_mx[0] <= u_max)) ? 1.0 : 0.0;  // unstable flag
    }
}

hipError_t launch_diag(const LatDesc* d, const double* fields, double* part, double* out, int ny,
                       double step, double u_max, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_rows, dim3(ny), dim3(256), 0, s, d, fields, part);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, s, d, fields, part, out, step, u_max);
    return hipGetLastError();
}

// Per-row sums use "y phi" through the row index: sum_y y * (sum_x phi) equals sum y phi.

// ------------------------------------------------------------ copy kernel

// Four independent 16-byte loads per lane before the stores, grid of 64
// workgroups per CU: the attainable device-to-device copy bandwidth.
__global__ void __launch_bounds__(256) k_copy(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                              int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * 1024;
    for (int64_t b = blockIdx.x * (int64_t)1024 + threadIdx.x; b < n16; b += stride) {
        uint4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = b + u * 256;
            v[u] = i < n16 ? src[i] : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = b + u * 256;
            if (i < n16) dst[i] = v[u];
        }
    }
}

// Both slots of a lattice's step counter (one thread; a kernel rather than a
// copy, so that it needs no host buffer and records no memset node in a graph).
__global__ void k_set_step(uint32_t* __restrict__ tstep, uint32_t t) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        tstep[0] = t;
        tstep[1] = t;
    }
}

hipError_t launch_set_step(uint32_t* tstep, uint32_t t, hipStream_t s) {
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, s, tstep, t);
    return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, uint64_t n, hipStream_t s) {
    const int64_t n16 = (int64_t)(n / 16);
    int64_t g = (n16 + 1023) / 1024;
    if (g > 256 * 64) g = 256 * 64;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_copy, dim3((int)g), dim3(256), 0, s, (uint4*)dst, (const uint4*)src, n16);
    return hipGetLastError();
}

// ------------------------------------------------- bandwidth probe variants
//
// Streams of 16-byte words that bound what the step kernel can reach: copies
// (one read and one write per word, the step's 1:1 mix) with more loads in flight,
// nontemporal accesses, or one contiguous chunk per workgroup; and pure reads
// and pure writes.  U unrolled words per lane are loaded before any is stored.

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int U, bool NT_LOAD, bool NT_STORE>
__global__ void __launch_bounds__(256) k_copy_strided(u32x4* __restrict__ dst, const u32x4* __restrict__ src,
                                                      int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * 256 * U;
    for (int64_t b = blockIdx.x * (int64_t)256 * U + threadIdx.x; b < n16; b += stride) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = b + u * 256;
            if (i < n16) v[u] = NT_LOAD ? __builtin_nontemporal_load(src + i) : src[i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = b + u * 256;
            if (i < n16) {
                if (NT_STORE) __builtin_nontemporal_store(v[u], dst + i);
                else dst[i] = v[u];
            }
        }
    }
}

// Each workgroup copies one contiguous chunk of the array (chunk words, a
// multiple of 256 U), U words per lane in flight.
template <int U>
__global__ void __launch_bounds__(256) k_copy_chunked(u32x4* __restrict__ dst, const u32x4* __restrict__ src,
                                                      int64_t n16, int64_t chunk) {
    const int64_t b0 = blockIdx.x * chunk, b1 = min(n16, b0 + chunk);
    for (int64_t b = b0 + threadIdx.x; b < b1; b += 256 * U) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = b + u * 256;
            if (i < b1) v[u] = src[i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = b + u * 256;
            if (i < b1) dst[i] = v[u];
        }
    }
}

// Reads every word (XOR-folded in registers), then writes one word per lane:
// the read bandwidth.
template <int U>
__global__ void __launch_bounds__(256) k_read_only(u32x4* __restrict__ out, const u32x4* __restrict__ src,
                                                   int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * 256 * U;
    u32x4 acc = {0u, 0u, 0u, 0u};
    for (int64_t b = blockIdx.x * (int64_t)256 * U + threadIdx.x; b < n16; b += stride) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = b + u * 256;
            if (i < n16) acc ^= src[i];
        }
    }
    out[blockIdx.x * 256 + threadIdx.x] = acc;
}

// Writes every word (its index in the first component): the write bandwidth.
template <int U>
__global__ void __launch_bounds__(256) k_write_only(u32x4* __restrict__ dst, int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * 256 * U;
    for (int64_t b = blockIdx.x * (int64_t)256 * U + threadIdx.x; b < n16; b += stride) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = b + u * 256;
            if (i < n16) {
                u32x4 v = {(unsigned)i, 0u, 0u, 0u};
                dst[i] = v;
            }
        }
    }
}

// The step kernel's memory pattern without its arithmetic: rows of 18 planes of
// 16-bit values, kRowCols columns each (18 strips of 448), a grid of 18 strips x
// 28 row segments (two workgroups per CU).  Per row a lane loads its 18 values,
// then stores them: one column per lane with 2-byte accesses (W2 false, 448
// lanes), or two columns per lane with 4-byte accesses (W2 true, 224 lanes).
constexpr int kRowCols = 8064, kRowStrips = 18, kRowSegs = 28;
template <bool W2>
__global__ void __launch_bounds__(448) k_rows16(uint16_t* __restrict__ dst, const uint16_t* __restrict__ src,
                                                int rows) {
    const int strip = blockIdx.x % kRowStrips, seg = blockIdx.x / kRowStrips;
    const int per = (rows + kRowSegs - 1) / kRowSegs;
    const int r0 = seg * per, r1 = min(rows, r0 + per);
    const uint32_t col = (uint32_t)(strip * 448 + (W2 ? 2 : 1) * (int)threadIdx.x);
    const uint32_t P = kRowCols * 2;  // bytes per plane
    for (int r = r0; r < r1; ++r) {
        const auto rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(src) + (size_t)r * 18 * kRowCols,
                                                          (short)0, -1, 0x00020000);
        const auto rd = __builtin_amdgcn_make_buffer_rsrc(dst + (size_t)r * 18 * kRowCols, (short)0, -1, 0x00020000);
        if constexpr (W2) {
            uint32_t v[18];
#pragma unroll
            for (int q = 0; q < 18; ++q) v[q] = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)(col * 2), (int)(q * P), 0);
#pragma unroll
            for (int q = 0; q < 18; ++q) __builtin_amdgcn_raw_buffer_store_b32(v[q] ^ 1u, rd, (int)(col * 2), (int)(q * P), 0);
        } else {
            uint16_t v[18];
#pragma unroll
            for (int q = 0; q < 18; ++q) v[q] = __builtin_amdgcn_raw_buffer_load_b16(rs, (int)(col * 2), (int)(q * P), 0);
#pragma unroll
            for (int q = 0; q < 18; ++q)
                __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(v[q] ^ 1u), rd, (int)(col * 2), (int)(q * P), 0);
        }
    }
}

hipError_t launch_bandwidth_probe(void* dst, const void* src, uint64_t n, int variant, hipStream_t s) {
    const int64_t n16 = (int64_t)(n / 16);
    if (n16 < 256 * 8) return hipErrorInvalidValue;
    u32x4* d = (u32x4*)dst;
    const u32x4* c = (const u32x4*)src;
    const int grid = 256 * 16;  // persistent: 16 workgroups of 256 lanes per CU
    switch (variant) {
    case 0: return launch_copy(dst, src, n, s);
    case 1: hipLaunchKernelGGL((k_copy_strided<8, false, false>), dim3(grid), dim3(256), 0, s, d, c, n16); break;
    case 2: hipLaunchKernelGGL((k_copy_strided<8, true, true>), dim3(grid), dim3(256), 0, s, d, c, n16); break;
    case 3: hipLaunchKernelGGL((k_copy_strided<4, false, true>), dim3(grid), dim3(256), 0, s, d, c, n16); break;
    case 4: {
        const int g = 256 * 8;
        int64_t chunk = (n16 + g - 1) / g;
        chunk = (chunk + 2047) / 2048 * 2048;
        hipLaunchKernelGGL((k_copy_chunked<8>), dim3((unsigned)((n16 + chunk - 1) / chunk)), dim3(256), 0, s, d, c,
                           n16, chunk);
        break;
    }
    case 5:
        // out: one word per lane of the grid, 16 MiB (n >= 4096 * 256 * 16 bytes is required)
        if (n16 < (int64_t)grid * 256) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_read_only<8>), dim3(grid), dim3(256), 0, s, d, c, n16);
        break;
    case 6: hipLaunchKernelGGL((k_write_only<8>), dim3(grid), dim3(256), 0, s, d, n16); break;
    case 7:
    case 8: {
        const int rows = (int)(n / (18ull * kRowCols * 2));
        if (rows < kRowSegs) return hipErrorInvalidValue;
        if (variant == 7)
            hipLaunchKernelGGL((k_rows16<false>), dim3(kRowStrips * kRowSegs), dim3(448), 0, s, (uint16_t*)dst,
                               (const uint16_t*)src, rows);
        else
            hipLaunchKernelGGL((k_rows16<true>), dim3(kRowStrips * kRowSegs), dim3(224), 0, s, (uint16_t*)dst,
                               (const uint16_t*)src, rows);
        break;
    }
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace cmlb
