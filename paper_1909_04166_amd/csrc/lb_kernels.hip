// lb_kernels.hip -- kernel instantiations and launchers (gfx950).
#include "lb_internal.hpp"

namespace cmlb {

// ------------------------------------------------------------ fused step

template <class ST, int MODE, bool PF>
static hipError_t launch_fused_tx(int tx, const LatDesc* d, const WorkItem* items, int n_items,
                                  int grid, int parity, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (grid <= 0 || grid > n_items) grid = n_items;
    switch (tx) {
    case 64: hipLaunchKernelGGL((lb_fused<ST, 64, MODE, PF>), dim3(grid), dim3(64), 0, s, d, items, n_items, parity); break;
    case 128: hipLaunchKernelGGL((lb_fused<ST, 128, MODE, PF>), dim3(grid), dim3(128), 0, s, d, items, n_items, parity); break;
    case 256: hipLaunchKernelGGL((lb_fused<ST, 256, MODE, PF>), dim3(grid), dim3(256), 0, s, d, items, n_items, parity); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class ST>
static hipError_t launch_step_st(int tx, int pf, const LatDesc* d, const WorkItem* items, int n_items,
                                 int grid, int parity, hipStream_t s) {
    return pf ? launch_fused_tx<ST, MODE_STEP, true>(tx, d, items, n_items, grid, parity, s)
              : launch_fused_tx<ST, MODE_STEP, false>(tx, d, items, n_items, grid, parity, s);
}

hipError_t launch_step(int prec, int tx, int pf, const LatDesc* d, const WorkItem* items, int n_items,
                       int grid, int parity, hipStream_t s) {
    switch (prec) {
    case LB_FP64: return launch_step_st<StF64>(tx, pf, d, items, n_items, grid, parity, s);
    case LB_FP32: return launch_step_st<StF32>(tx, pf, d, items, n_items, grid, parity, s);
    case LB_FP32_F16: return launch_step_st<StF16>(tx, pf, d, items, n_items, grid, parity, s);
    case LB_FP32_BF16: return launch_step_st<StBF16>(tx, pf, d, items, n_items, grid, parity, s);
    }
    return hipErrorInvalidValue;
}

template <class ST, bool PF>
static int occ_tx(int tx) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (tx) {
    case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lb_fused<ST, 64, MODE_STEP, PF>, 64, 0); break;
    case 128: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lb_fused<ST, 128, MODE_STEP, PF>, 128, 0); break;
    case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lb_fused<ST, 256, MODE_STEP, PF>, 256, 0); break;
    }
    return e == hipSuccess ? nb : 1;
}

int fused_occupancy(int prec, int tx, int pf) {
    switch (prec) {
    case LB_FP64: return pf ? occ_tx<StF64, true>(tx) : occ_tx<StF64, false>(tx);
    case LB_FP32: return pf ? occ_tx<StF32, true>(tx) : occ_tx<StF32, false>(tx);
    case LB_FP32_F16: return pf ? occ_tx<StF16, true>(tx) : occ_tx<StF16, false>(tx);
    case LB_FP32_BF16: return pf ? occ_tx<StBF16, true>(tx) : occ_tx<StBF16, false>(tx);
    }
    return 1;
}

// Fields / coupling extraction always runs with 64-wide strips.
hipError_t launch_extract(int prec, int mode, const LatDesc* d, const WorkItem* items64,
                          int n_items, int parity, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
#define CMLB_EXTRACT(ST)                                                                          \
    if (mode == MODE_FIELDS)                                                                      \
        hipLaunchKernelGGL((lb_fused<ST, 64, MODE_FIELDS, false>), dim3(n_items), dim3(64), 0, s, d,   \
                           items64, n_items, parity);                                             \
    else                                                                                          \
        hipLaunchKernelGGL((lb_fused<ST, 64, MODE_COUPLING, false>), dim3(n_items), dim3(64), 0, s, d, \
                           items64, n_items, parity);
    switch (prec) {
    case LB_FP64: CMLB_EXTRACT(StF64); break;
    case LB_FP32: CMLB_EXTRACT(StF32); break;
    case LB_FP32_F16: CMLB_EXTRACT(StF16); break;
    case LB_FP32_BF16: CMLB_EXTRACT(StBF16); break;
    default: return hipErrorInvalidValue;
    }
#undef CMLB_EXTRACT
    return hipGetLastError();
}

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

// Stored (pre-streaming) value of direction a at node (x, y) such that pulling
// gives the post-streaming value val(b, x', y'):  f~_a(x) = f_a(x + e_a), or
// f_{opp a}(x) when x + e_a lies beyond a halfway wall.
// The state at t = 0 is f_a = w_a phi0, gbar_a = 0.
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
            int xs = x + ex_of(a), ys = y + ey_of(a);
            xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
            double ph;
            if (ys < 0 || ys >= ny) {
                if (D.wall_y) ph = phi0[k];  // f_{opp a}(x) = w phi0(x), w_opp = w_a
                else ph = phi0[(int64_t)(ys < 0 ? ys + ny : ys - ny) * nx + xs];
            } else {
                ph = phi0[(int64_t)ys * nx + xs];
            }
            const double w = wgt(a);
            buf[a * D.plane + k] = ST::st((typename ST::R)(w * ph - w * D.shift_f));
            buf[(9 + a) * D.plane + k] = ST::st((typename ST::R)(0.0 - w * D.shift_g));
        }
    }
}

// Writes the stored planes from one staged post-streaming FP64 plane b of f
// (which = 0) or gbar (which = 1): f~_b(x) = f_b(x + e_b) where x + e_b is inside,
// and f~_{opp b}(x) = f_b(x) where x - e_b lies beyond a wall.
template <class ST>
__global__ void k_set_plane(const LatDesc* __restrict__ dp, const double* __restrict__ stage,
                            int b, int which, int cur) {
    const LatDesc& D = *dp;
    const int nx = D.nx, ny = D.ny;
    const int64_t N = (int64_t)nx * ny;
    using T = typename ST::T;
    T* buf = reinterpret_cast<T*>(D.buf[cur]) + (which ? 9 * D.plane : 0);
    const double sh = which ? D.shift_g : D.shift_f;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < N;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(k / nx), x = (int)(k % nx);
        int xs = x + ex_of(b), ys = y + ey_of(b);
        xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
        const bool out = ys < 0 || ys >= ny;
        if (!out || !D.wall_y) {
            if (out) ys = ys < 0 ? ys + ny : ys - ny;
            buf[b * D.plane + k] = ST::st((typename ST::R)(stage[(int64_t)ys * nx + xs] - wgt(b) * sh));
        }
        const int yb = y - ey_of(b);
        if (D.wall_y && (yb < 0 || yb >= ny)) {
            const int o = opp_of(b);
            buf[o * D.plane + k] = ST::st((typename ST::R)(stage[k] - wgt(o) * sh));
        }
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
    const T* buf = reinterpret_cast<const T*>(D.buf[cur]) + (which ? 9 * D.plane : 0);
    const double sh = which ? D.shift_g : D.shift_f;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < N;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(k / nx), x = (int)(k % nx);
        int xs = x - ex_of(a), ys = y - ey_of(a);
        xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
        const bool outside = ys < 0 || ys >= ny;
        double v;
        if (outside && D.wall_y) {
            const int o = opp_of(a);
            v = (double)ST::ld(buf[o * D.plane + k]) + wgt(o) * sh;
        } else {
            if (outside) ys = ys < 0 ? ys + ny : ys - ny;
            v = (double)ST::ld(buf[a * D.plane + (int64_t)ys * nx + xs]) + wgt(a) * sh;
        }
        out[k] = v;
    }
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
        if (!(um <= mx)) mx = um;
        if (!isfinite(ph) || !isfinite(p) || !isfinite(um)) nn += 1;
    }
    s_phi[threadIdx.x] = sp; s_rho[threadIdx.x] = sr; s_max[threadIdx.x] = mx; s_nan[threadIdx.x] = nn;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            s_phi[threadIdx.x] += s_phi[threadIdx.x + st];
            s_rho[threadIdx.x] += s_rho[threadIdx.x + st];
            const double o = s_max[threadIdx.x + st];
            if (!(o <= s_max[threadIdx.x])) s_max[threadIdx.x] = o;
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

__device__ double crossing_dev(const double* phi, int nx, int ny, int x, int dir) {
    if (dir > 0) {
        for (int j = 0; j + 1 < ny; ++j) {
            const double a = phi[(int64_t)j * nx + x] - 0.5, b = phi[(int64_t)(j + 1) * nx + x] - 0.5;
            if ((a < 0) != (b < 0)) return j + a / (a - b);
        }
    } else {
        for (int j = ny - 2; j >= 0; --j) {
            const double a = phi[(int64_t)j * nx + x] - 0.5, b = phi[(int64_t)(j + 1) * nx + x] - 0.5;
            if ((a < 0) != (b < 0)) return j + a / (a - b);
        }
    }
    return __longlong_as_double(0x7ff8000000000000LL);
}

// Final pass: rows summed in order by one thread; tips scanned by two threads.
__global__ void k_diag_final(const LatDesc* __restrict__ dp, const double* __restrict__ F,
                             const double* __restrict__ part, double* __restrict__ out,
                             double step, double u_max) {
    const LatDesc& D = *dp;
    const int nx = D.nx, ny = D.ny;
    const int64_t N = (int64_t)nx * ny;
    if (threadIdx.x == 0) {
        double sp = 0, sr = 0, sy = 0, mx = 0, nn = 0;
        for (int y = 0; y < ny; ++y) {
            sp += part[4 * (int64_t)y];
            sr += part[4 * (int64_t)y + 1];
            sy += (double)y * part[4 * (int64_t)y];
            const double o = part[4 * (int64_t)y + 2];
            if (!(o <= mx)) mx = o;
            nn += part[4 * (int64_t)y + 3];
        }
        out[0] = step;
        out[1] = sp;
        out[2] = sr;
        out[3] = mx;
        out[4] = F[N + (int64_t)(ny / 2) * nx + nx / 2] - F[N];
        out[5] = sqrt(sp / 3.14159265358979323846);
        out[8] = sy / sp;
        out[9] = nn > 0 ? 1.0 : 0.0;
        out[10] = (nn > 0 || !(mx <= u_max)) ? 1.0 : 0.0;  // unstable flag
    } else if (threadIdx.x == 1) {
        out[6] = crossing_dev(F, nx, ny, nx / 2, +1);
    } else if (threadIdx.x == 2) {
        out[7] = crossing_dev(F, nx, ny, 0, -1);
    }
}

hipError_t launch_diag(const LatDesc* d, const double* fields, double* part, double* out, int ny,
                       double step, double u_max, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_rows, dim3(ny), dim3(256), 0, s, d, fields, part);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, s, d, fields, part, out, step, u_max);
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

hipError_t launch_copy(void* dst, const void* src, uint64_t n, hipStream_t s) {
    const int64_t n16 = (int64_t)(n / 16);
    int64_t g = (n16 + 1023) / 1024;
    if (g > 256 * 64) g = 256 * 64;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_copy, dim3((int)g), dim3(256), 0, s, (uint4*)dst, (const uint4*)src, n16);
    return hipGetLastError();
}

}  // namespace cmlb
