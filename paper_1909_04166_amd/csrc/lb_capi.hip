// lb_capi.hip -- host runtime behind the C-ABI of include/cmlb.h: parameter
// validation, workspace layout, work lists, stepping (eager or replayed HIP
// graphs), diagnostics, checkpoints, the batch of uneven lattices with its node
// pool, and the tile autotuner.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "lb_internal.hpp"

using namespace cmlb;

namespace {

// A roctx range over one host call (lb_step, lb_batch_step): a marker trace
// (rocprofv3 --marker-trace) shows each call around the kernels it launches.
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
};

constexpr uint64_t kAlign = 256;
constexpr int kMinH = 1;
// Nontemporal stores only for states well above the 256 MB last-level cache
// (MALL): a smaller state stays there between steps, and streaming its stores
// past it made the 75 MB Rayleigh-Taylor lattice 13% slower.
constexpr uint64_t kStreamBytes = (uint64_t)1 << 30;
// A batch replays captured step graphs once its work list has been unchanged for
// this many graph lengths (steps).
constexpr int kGraphAfter = 4;

uint64_t align_up(uint64_t v, uint64_t a = kAlign) { return (v + a - 1) / a * a; }

int store_bytes(int prec) {
    switch (prec) {
    case LB_FP64: return 8;
    case LB_FP32: return 4;
    case LB_FP32_F16:
    case LB_FP32_BF16: return 2;
    }
    return 0;
}

int64_t plane_elems(int nx, int ny) { return (int64_t)align_up((uint64_t)nx * ny, 64); }

bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

// Workgroup widths with a step kernel: powers of two, 64k + 4 (strips of whole
// 64-column blocks: 132, 260, 516, and 452 = two 8-wave workgroups per CU at four
// waves per SIMD), and 1024 (16 waves per CU: FP32-compute kernels without
// prefetching only).
bool valid_width(int tx, int prec, int pf) {
    switch (tx) {
    case 64: case 128: case 132: case 256: case 260: case 452: case 512: case 516: return true;
    case 1024: return prec != LB_FP64 && pf == 0;
    }
    return false;
}

lb_status validate(const lb_config* c) {
    if (!c) return LB_E_INVALID_ARG;
    if (c->nx < 8 || c->ny < 8 || c->nx > (1 << 20) || c->ny > (1 << 20)) return LB_E_INVALID_ARG;
    // every plane (storage type) and every FP64 field plane must be < 4 GiB
    if ((uint64_t)c->nx * c->ny * 8 >= ((uint64_t)1 << 32)) return LB_E_INVALID_ARG;
    if (c->bc_x != LB_PERIODIC && c->bc_x != LB_HALFWAY_BB && c->bc_x != LB_FREE_SLIP)
        return LB_E_INVALID_ARG;
    if (c->bc_y != LB_PERIODIC && c->bc_y != LB_HALFWAY_BB && c->bc_y != LB_FREE_SLIP)
        return LB_E_INVALID_ARG;
    if (c->collision != LB_CASCADED && c->collision != LB_SRT && c->collision != LB_CASCADED_PRINTED)
        return LB_E_INVALID_ARG;
    if (c->flow != LB_FLOW_COUPLED && c->flow != LB_FLOW_IMPOSED) return LB_E_INVALID_ARG;
    if (c->surf != LB_SIGMA_LINEAR && c->surf != LB_SIGMA_LANGMUIR) return LB_E_INVALID_ARG;
    if (c->tile_pf < 0 || c->tile_pf > 1) return LB_E_INVALID_ARG;
    if (c->tile_pf != 0 && (c->tile_x == 0 || c->tile_h == 0 || c->collision != LB_CASCADED ||
                            c->flow != LB_FLOW_COUPLED))
        return LB_E_INVALID_ARG;
    if (c->force_ref < LB_FREF_MEAN || c->force_ref > LB_FREF_NONE) return LB_E_INVALID_ARG;
    if (c->st_form != LB_ST_GEOMETRIC && c->st_form != LB_ST_CHEMPOT) return LB_E_INVALID_ARG;
    if (store_bytes(c->precision) == 0) return LB_E_INVALID_ARG;
    if (!finite_pos(c->rho_A) || !finite_pos(c->rho_B) || !finite_pos(c->nu_A) ||
        !finite_pos(c->nu_B) || !finite_pos(c->W) || !finite_pos(c->M))
        return LB_E_INVALID_ARG;
    const double vals[] = {c->sigma0, c->sigma_T, c->T0, c->dTdy, c->y_ref, c->gx, c->gy,
                           c->shift_f, c->shift_g, c->u_max, c->beta, c->psi_a, c->psi_G};
    for (double v : vals)
        if (!std::isfinite(v)) return LB_E_INVALID_ARG;
    if (c->surf == LB_SIGMA_LANGMUIR) {
        if (c->st_form != LB_ST_GEOMETRIC) return LB_E_UNSUPPORTED;
        // 1 - psi(y) > 0 on every row (psi is linear: check the end rows)
        if (!(1.0 - c->psi_a > 0.0) || !(1.0 - (c->psi_a + c->psi_G * (c->ny - 1)) > 0.0))
            return LB_E_INVALID_ARG;
    }
    // derived rates in (0, 2): omega_nu = 1/(1/2 + 3 nu) at both phases, omega_phi
    const double om[] = {1.0 / (0.5 + 3.0 * c->nu_A), 1.0 / (0.5 + 3.0 * c->nu_B),
                         1.0 / (0.5 + 3.0 * c->M)};
    for (double o : om)
        if (!(o > 0.0 && o < 2.0)) return LB_E_INVALID_ARG;
    if (c->tile_x != 0 && !valid_width(c->tile_x, c->precision, c->tile_pf)) return LB_E_INVALID_ARG;
    if (c->tile_h < 0 || (c->tile_h > 0 && c->tile_h < kMinH)) return LB_E_INVALID_ARG;
    if (c->diag_every < 0) return LB_E_INVALID_ARG;
    if (c->init_kind < LB_INIT_NONE || c->init_kind > LB_INIT_INTERFACE) return LB_E_INVALID_ARG;
    if (c->rounding != LB_ROUND_STOCHASTIC && c->rounding != LB_ROUND_NEAREST) return LB_E_INVALID_ARG;
    for (double v : c->init_par)
        if (!std::isfinite(v)) return LB_E_INVALID_ARG;
    if (c->init_kind == LB_INIT_DROPLET &&
        (!(c->init_par[2] > 0) || std::fabs(c->init_par[3]) != 1.0 || c->init_par[4] < 0 || c->init_par[5] < 0))
        return LB_E_INVALID_ARG;
    if (c->init_kind == LB_INIT_ELLIPSE &&
        (!(c->init_par[2] > 0) || !(c->init_par[3] > 0) || c->init_par[4] < 0 || c->init_par[5] < 0))
        return LB_E_INVALID_ARG;
    return LB_OK;
}

double rho_ref_of(const lb_config* c) {
    switch (c->force_ref) {
    case LB_FREF_LIGHT: return std::min(c->rho_A, c->rho_B);
    case LB_FREF_HEAVY: return std::max(c->rho_A, c->rho_B);
    case LB_FREF_NONE: return 0.0;
    default: return 0.5 * (c->rho_A + c->rho_B);
    }
}

int kind_of(const lb_config* c) {
    const bool srt = c->collision == LB_SRT;
    if (c->flow == LB_FLOW_IMPOSED) return srt ? KIND_ACE_SRT : KIND_ACE_CASCADED;  // one phase-field cascade
    if (c->collision == LB_CASCADED_PRINTED) return KIND_COUPLED_PRINTED;
    return srt ? KIND_COUPLED_SRT : KIND_COUPLED_CASCADED;
}

void fill_desc(const lb_config* c, LatDesc& D, void* b0, void* b1, int64_t plane, double* fields) {
    std::memset(&D, 0, sizeof(D));
    D.nx = c->nx;
    D.ny = c->ny;
    D.wall_y = c->bc_y == LB_HALFWAY_BB ? WALL_BOUNCE : (c->bc_y == LB_FREE_SLIP ? WALL_SLIP : WALL_NONE);
    D.wall_x = c->bc_x == LB_HALFWAY_BB ? WALL_BOUNCE : (c->bc_x == LB_FREE_SLIP ? WALL_SLIP : WALL_NONE);
    D.st_form = c->st_form;
    D.surf = c->surf == LB_SIGMA_LANGMUIR ? 1 : 0;
    D.flow = c->flow == LB_FLOW_IMPOSED ? 1 : 0;
    D.plane = plane;
    D.buf[0] = b0;
    D.buf[1] = b1;
    D.fields = fields;
    D.rhoB = c->rho_B;
    D.dRho = c->rho_A - c->rho_B;
    const double muA = c->rho_A * c->nu_A, muB = c->rho_B * c->nu_B;
    D.muB = muB;
    D.dMu = muA - muB;
    // sigma(y) = s_a + s_b y
    const double s_a = c->sigma0 + c->sigma_T * (c->T0 - c->dTdy * c->y_ref);
    const double s_b = c->sigma_T * c->dTdy;
    D.kt_a = 1.5 * c->W * s_a;
    D.kt_b = 1.5 * c->W * s_b;
    D.be_a = 12.0 * s_a / c->W;
    D.be_b = 12.0 * s_b / c->W;
    D.ka_a = 1.5 * c->W * s_a;
    D.ka_b = 1.5 * c->W * s_b;
    D.four_W = 4.0 / c->W;
    D.M = c->M;
    D.omphi = 1.0 / (0.5 + 3.0 * c->M);
    D.gx = c->gx;
    D.gy = c->gy;
    D.rho_ref = rho_ref_of(c);
    const bool half = c->precision == LB_FP32_F16 || c->precision == LB_FP32_BF16;
    D.shift_f = half ? c->shift_f : 0.0;
    D.shift_g = half ? c->shift_g : 0.0;
    D.sround = half && c->rounding == LB_ROUND_STOCHASTIC ? 1 : 0;
    D.ntstore = ((int64_t)c->nx * store_bytes(c->precision)) % 128 == 0 ? 1 : 0;
    D.kt0 = 1.5 * c->W * c->sigma0;
    D.lbeta = c->beta;
    D.ps_a = c->psi_a;
    D.ps_G = c->psi_G;
}

int max_items_for(int nx, int ny) {
    return ((nx + 59) / 60) * ((ny + kMinH - 1) / kMinH) + 3 * kMaxGrid;
}

int cu_count() {
    static int n = -1;
    if (n < 0) {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
            n = p.multiProcessorCount;
        else
            n = 256;
    }
    return n;
}

bool build_schedule(const std::vector<LatShape>& lats, int prec, int kind, bool walls, Sched& sc, int max_items,
                    std::vector<WorkItem>& items) {
    const int resident = sc.mode == 0 ? 1 : step_occupancy(prec, kind, walls, sc.tx, sc.pf);
    return plan_schedule(lats, resident, cu_count(), sc, max_items, items);
}

// The schedule of lattices too small to autotune and of lb_step_noalloc
// (lb_sched.hpp), prefetching where the kernel has it.
Sched default_sched(int nx, int ny, int kind) {
    return small_lattice_sched(nx, ny, kind == KIND_COUPLED_CASCADED, cu_count(), kMinH);
}

struct TuneKey {
    int prec, nx, ny, wall, wallx, st, kind, surf;
    bool operator<(const TuneKey& o) const {
        return std::tie(prec, nx, ny, wall, wallx, st, kind, surf) <
               std::tie(o.prec, o.nx, o.ny, o.wall, o.wallx, o.st, o.kind, o.surf);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, Sched> g_tune;

#define HIPC(x)                                 \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return LB_E_HIP;  \
    } while (0)

}  // namespace

// ======================================================================== single

struct lb_handle {
    lb_config cfg;
    int kind = KIND_COUPLED_CASCADED;
    bool walls = true;  // the lattice has a wall on some side (else the wall-free kernels run)
    bool nt = false;    // its rows are whole cache lines and its state is large (nontemporal stores
                        // where the strips are whole lines too)
    hipStream_t s = nullptr;
    char* ws = nullptr;
    uint64_t ws_bytes = 0;
    LatDesc hdesc;
    LatDesc* d_desc = nullptr;     // fields -> d_fields
    LatDesc* d_desc_cp = nullptr;  // fields -> caller buffer (coupling output)
    WorkItem* d_items = nullptr;
    int n_items = 0, max_items = 0;
    WorkItem* d_items64 = nullptr;
    int n_items64 = 0;
    double* d_part = nullptr;
    double* d_dout = nullptr;
    double* d_fields = nullptr;
    void* buf[2] = {nullptr, nullptr};
    int64_t plane = 0;
    int sbytes = 0;
    int parity = 0;
    int64_t step = 0;
    Sched sc;
    bool tuned = false;
    // diagnostics
    double* h_diag = nullptr;  // pinned, 16 doubles
    hipEvent_t ev_diag = nullptr;
    bool diag_pending = false;
    bool unstable = false;
    // timing
    bool timing = false;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    int64_t last_steps = 0;
    // graphs: one per starting parity
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int glen = 0;
};

namespace {

struct Layout {
    uint64_t desc, desc_cp, tstep, items, items64, part, dout, fields, bufA, bufB, vel, ktab, total;
};

Layout layout_of(const lb_config* c) {
    Layout L;
    const int64_t N = (int64_t)c->nx * c->ny;
    const int64_t P = plane_elems(c->nx, c->ny);
    const int sb = store_bytes(c->precision);
    uint64_t o = 0;
    L.desc = o; o += align_up(sizeof(LatDesc));
    L.desc_cp = o; o += align_up(sizeof(LatDesc));
    L.tstep = o; o += align_up(2 * sizeof(uint32_t));
    L.items = o; o += align_up((uint64_t)max_items_for(c->nx, c->ny) * sizeof(WorkItem));
    L.items64 = o; o += align_up((uint64_t)((c->nx + 59) / 60) * ((c->ny + 63) / 64) * sizeof(WorkItem));
    L.part = o; o += align_up((uint64_t)4 * c->ny * sizeof(double));
    L.dout = o; o += align_up(16 * sizeof(double));
    L.fields = o; o += align_up((uint64_t)4 * N * sizeof(double));
    L.bufA = o; o += align_up((uint64_t)18 * P * sb);
    L.bufB = o; o += align_up((uint64_t)18 * P * sb);
    L.vel = o;
    if (c->flow == LB_FLOW_IMPOSED) o += align_up((uint64_t)2 * P * (c->precision == LB_FP64 ? 8 : 4));
    L.ktab = o; o += align_up((uint64_t)2 * c->ny * sizeof(double));
    L.total = o;
    return L;
}

lb_status set_sched(lb_handle* h, Sched sc) {
    std::vector<WorkItem> items;
    if (!build_schedule({{0, h->cfg.nx, h->cfg.ny}}, h->cfg.precision, h->kind, h->walls, sc, h->max_items, items))
        return LB_E_INVALID_ARG;
    HIPC(hipMemcpyAsync(h->d_items, items.data(), items.size() * sizeof(WorkItem),
                        hipMemcpyHostToDevice, h->s));
    HIPC(hipStreamSynchronize(h->s));
    h->n_items = sc.n_items;
    h->sc = sc;
    for (int p = 0; p < 2; ++p)
        if (h->gexec[p]) { (void)hipGraphExecDestroy(h->gexec[p]); h->gexec[p] = nullptr; }
    return LB_OK;
}

lb_status launch_steps_eager(lb_handle* h, int64_t n) {
    for (int64_t i = 0; i < n; ++i) {
        HIPC(launch_step(h->cfg.precision, h->kind, h->walls, h->nt, h->sc.tx, h->sc.pf, h->d_desc, h->d_items, h->n_items,
                         h->sc.grid, h->parity, h->s));
        h->parity ^= 1;
        h->step += 1;
    }
    return LB_OK;
}

// Replays a captured graph of glen steps (glen even, so the parity is restored).
lb_status graph_for(lb_handle* h, int parity, hipGraphExec_t* out) {
    if (!h->gexec[parity]) {
        hipStream_t cs;
        HIPC(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        int p = parity;
        for (int i = 0; i < h->glen && e == hipSuccess; ++i) {
            e = launch_step(h->cfg.precision, h->kind, h->walls, h->nt, h->sc.tx, h->sc.pf, h->d_desc, h->d_items, h->n_items,
                            h->sc.grid, p, cs);
            p ^= 1;
        }
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess || e2 != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return LB_E_HIP;
        }
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return LB_E_HIP;
        h->gexec[parity] = ex;
    }
    *out = h->gexec[parity];
    return LB_OK;
}

lb_status enqueue_diag(lb_handle* h) {
    HIPC(launch_extract(h->cfg.precision, h->kind, MODE_FIELDS, h->d_desc, h->d_items64, h->n_items64,
                        h->parity, h->s));
    const double umax = h->cfg.u_max > 0 ? h->cfg.u_max : 0.3;
    HIPC(launch_diag(h->d_desc, h->d_fields, h->d_part, h->d_dout, h->cfg.ny, (double)h->step,
                     umax, h->s));
    return LB_OK;
}

// Times `reps` launches of one candidate without advancing the state (every
// launch reads the current buffer and overwrites the other one).
double time_candidate(int prec, int kind, bool walls, bool nt, int tx, int pf, const LatDesc* d, const WorkItem* items, int n,
                      int grid, int parity, hipStream_t s, int reps) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return 1e30;
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return 1e30; }
    double ms_out = 1e30;
    bool ok = launch_step(prec, kind, walls, nt, tx, pf, d, items, n, grid, parity, s) == hipSuccess;
    ok = ok && hipEventRecord(a, s) == hipSuccess;
    for (int i = 0; i < reps && ok; ++i)
        ok = launch_step(prec, kind, walls, nt, tx, pf, d, items, n, grid, parity, s) == hipSuccess;
    ok = ok && hipEventRecord(b, s) == hipSuccess && hipEventSynchronize(b) == hipSuccess;
    float ms = 0;
    if (ok && hipEventElapsedTime(&ms, a, b) == hipSuccess) ms_out = ms / reps;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms_out;
}

// Candidate schedules for one lattice shape (the prefetching variant exists for
// the coupled cascaded kernel only).
std::vector<Sched> candidates(int prec, int nx, int ny, int kind) {
    std::vector<Sched> out;
    for (int pf : {PF_HOLD, PF_PREFETCH})
        for (int tx : {64, 128, 132, 256, 260, 452, 512, 516, 1024}) {
            if (pf != PF_HOLD && kind != KIND_COUPLED_CASCADED) continue;
            if (!valid_width(tx, prec, pf)) continue;
            if (tx > 64 && nx <= strip_w(tx / 2)) continue;
            for (int th : {1, 2, 4, 8, 16, 32, 64, 128, 256}) {
                if (th > ny && th != 16) continue;
                Sched sc;
                sc.tx = tx; sc.th = th; sc.mode = 0; sc.pf = pf;
                out.push_back(sc);
            }
            for (int mode : {1, 2})
                for (int m : {1, 2}) {
                    Sched sc;
                    sc.tx = tx; sc.mode = mode; sc.mult = m; sc.pf = pf;
                    out.push_back(sc);
                }
        }
    return out;
}

// The finalists' times that lie within 1% of the fastest are taken as equal
// (repeated timings of one schedule spread about that much); among those the
// schedule with the fewest work items wins, as it re-reads the fewest halo rows,
// then the one without prefetching, then the narrower workgroup, then the lower
// mode and multiplier.  This keeps the choice the same from run to run when
// schedules tie.
Sched pick_final(const std::vector<std::pair<double, Sched>>& fin, const Sched& fallback) {
    double best = 1e30;
    for (const auto& f : fin) best = std::min(best, f.first);
    auto key = [](const Sched& c) { return std::make_tuple(c.n_items, c.pf, c.tx, c.mode, c.mult, c.th); };
    const Sched* pick = nullptr;
    for (const auto& f : fin)
        if (f.first <= 1.01 * best && (!pick || key(f.second) < key(*pick))) pick = &f.second;
    return pick ? *pick : fallback;
}

lb_status autotune_single(lb_handle* h) {
    const TuneKey key{h->cfg.precision, h->cfg.nx, h->cfg.ny, h->hdesc.wall_y, h->hdesc.wall_x,
                      h->cfg.st_form, h->kind, h->cfg.surf};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) return set_sched(h, it->second);
    }
    const int64_t N = (int64_t)h->cfg.nx * h->cfg.ny;
    const int reps = N >= (1 << 22) ? 3 : 10;
    auto timed = [&](Sched& sc, int r, double* ms) -> lb_status {
        std::vector<WorkItem> items;
        *ms = 1e30;
        if (!build_schedule({{0, h->cfg.nx, h->cfg.ny}}, h->cfg.precision, h->kind, h->walls, sc, h->max_items, items))
            return LB_OK;
        HIPC(hipMemcpyAsync(h->d_items, items.data(), items.size() * sizeof(WorkItem),
                            hipMemcpyHostToDevice, h->s));
        *ms = time_candidate(h->cfg.precision, h->kind, h->walls, h->nt, sc.tx, sc.pf, h->d_desc, h->d_items, sc.n_items,
                             sc.grid, h->parity, h->s, r);
        return LB_OK;
    };
    // every candidate once, then the three fastest again with 4x the repetitions,
    // so that near-equal schedules are not picked by timing noise
    std::vector<std::pair<double, Sched>> scored;
    for (Sched sc : candidates(h->cfg.precision, h->cfg.nx, h->cfg.ny, h->kind)) {
        double ms;
        const lb_status st = timed(sc, reps, &ms);
        if (st != LB_OK) return st;
        if (ms < 1e30) scored.push_back({ms, sc});
    }
    std::sort(scored.begin(), scored.end(),
              [](const std::pair<double, Sched>& a, const std::pair<double, Sched>& b) { return a.first < b.first; });
    std::vector<std::pair<double, Sched>> fin;
    for (size_t i = 0; i < scored.size() && i < 3; ++i) {
        double ms;
        const lb_status st = timed(scored[i].second, 4 * reps, &ms);
        if (st != LB_OK) return st;
        if (ms < 1e30) fin.push_back({ms, scored[i].second});
    }
    const Sched best_sc = pick_final(fin, h->sc);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = best_sc;
    }
    return set_sched(h, best_sc);
}

}  // namespace

extern "C" {

const char* lb_status_string(lb_status s) {
    switch (s) {
    case LB_OK: return "ok";
    case LB_E_INVALID_ARG: return "invalid argument";
    case LB_E_WORKSPACE: return "workspace too small, misaligned or exhausted";
    case LB_E_HIP: return "HIP runtime error";
    case LB_E_UNSTABLE: return "unstable: NaN/Inf or max|u| above the limit";
    case LB_E_UNSUPPORTED: return "unsupported option";
    case LB_E_STATE: return "state buffer of the wrong size";
    case LB_E_TOO_LARGE: return "lattice too large for the 1 MiB static scratch of lb_step_noalloc";
    }
    return "unknown status";
}

lb_status lb_workspace_bytes(const lb_config* cfg, uint64_t* bytes) {
    if (!bytes) return LB_E_INVALID_ARG;
    lb_status st = validate(cfg);
    if (st != LB_OK) return st;
    *bytes = layout_of(cfg).total;
    return LB_OK;
}

lb_status lb_create(const lb_config* cfg, void* dev_ws, uint64_t ws_bytes, void* stream,
                    lb_handle** out) {
    if (!out || !dev_ws) return LB_E_INVALID_ARG;
    *out = nullptr;
    lb_status st = validate(cfg);
    if (st != LB_OK) return st;
    const Layout L = layout_of(cfg);
    if (ws_bytes < L.total || ((uintptr_t)dev_ws % kAlign)) return LB_E_WORKSPACE;
    lb_handle* h = new lb_handle();
    h->cfg = *cfg;
    h->s = (hipStream_t)stream;
    h->ws = (char*)dev_ws;
    h->ws_bytes = ws_bytes;
    h->d_desc = (LatDesc*)(h->ws + L.desc);
    h->d_desc_cp = (LatDesc*)(h->ws + L.desc_cp);
    h->d_items = (WorkItem*)(h->ws + L.items);
    h->max_items = max_items_for(cfg->nx, cfg->ny);
    h->d_items64 = (WorkItem*)(h->ws + L.items64);
    h->d_part = (double*)(h->ws + L.part);
    h->d_dout = (double*)(h->ws + L.dout);
    h->d_fields = (double*)(h->ws + L.fields);
    h->buf[0] = h->ws + L.bufA;
    h->buf[1] = h->ws + L.bufB;
    h->plane = plane_elems(cfg->nx, cfg->ny);
    h->sbytes = store_bytes(cfg->precision);
    h->glen = 32;
    h->kind = kind_of(cfg);
    fill_desc(cfg, h->hdesc, h->buf[0], h->buf[1], h->plane, h->d_fields);
    h->walls = h->hdesc.wall_y != WALL_NONE || h->hdesc.wall_x != WALL_NONE;
    h->nt = h->hdesc.ntstore != 0 && (uint64_t)2 * 18 * h->plane * h->sbytes >= kStreamBytes;
    h->hdesc.vel = cfg->flow == LB_FLOW_IMPOSED ? (void*)(h->ws + L.vel) : nullptr;
    h->hdesc.ktab = (double*)(h->ws + L.ktab);
    h->hdesc.tstep = (uint32_t*)(h->ws + L.tstep);
    auto fail = [&](lb_status s) { lb_destroy(h); return s; };
    if (hipHostMalloc((void**)&h->h_diag, 16 * sizeof(double), hipHostMallocDefault) != hipSuccess)
        return fail(LB_E_HIP);
    std::memset(h->h_diag, 0, 16 * sizeof(double));
    if (hipEventCreateWithFlags(&h->ev_diag, hipEventDisableTiming) != hipSuccess) return fail(LB_E_HIP);
    if (hipEventCreate(&h->t0) != hipSuccess || hipEventCreate(&h->t1) != hipSuccess)
        return fail(LB_E_HIP);
    if (hipMemcpyAsync(h->d_desc, &h->hdesc, sizeof(LatDesc), hipMemcpyHostToDevice, h->s) != hipSuccess)
        return fail(LB_E_HIP);
    if (launch_set_step(h->hdesc.tstep, 0, h->s) != hipSuccess) return fail(LB_E_HIP);
    if (cfg->surf == LB_SIGMA_LANGMUIR && launch_kappa_table(h->d_desc, cfg->ny, h->s) != hipSuccess)
        return fail(LB_E_HIP);
    // the imposed velocity is zero until lb_set_velocity
    if (h->hdesc.vel &&
        hipMemsetAsync(h->hdesc.vel, 0, L.ktab - L.vel, h->s) != hipSuccess)
        return fail(LB_E_HIP);
    std::vector<WorkItem> it64;
    build_items(0, cfg->nx, cfg->ny, 64, 64, it64);
    h->n_items64 = (int)it64.size();
    if (hipMemcpyAsync(h->d_items64, it64.data(), it64.size() * sizeof(WorkItem),
                       hipMemcpyHostToDevice, h->s) != hipSuccess)
        return fail(LB_E_HIP);
    Sched sc = default_sched(cfg->nx, cfg->ny, h->kind);
    if (cfg->tile_x) sc.tx = cfg->tile_x;
    if (cfg->tile_h) sc.th = cfg->tile_h;
    if (cfg->tile_x || cfg->tile_h) sc.pf = cfg->tile_pf;
    h->tuned = (cfg->tile_x != 0 && cfg->tile_h != 0) || (int64_t)cfg->nx * cfg->ny < (1 << 16);
    st = set_sched(h, sc);
    if (st != LB_OK) return fail(st);
    *out = h;
    return LB_OK;
}

lb_status lb_init_fields(lb_handle* h, const double* phi0) {
    if (!h || (!phi0 && h->cfg.init_kind == LB_INIT_NONE)) return LB_E_INVALID_ARG;
    const int64_t N = (int64_t)h->cfg.nx * h->cfg.ny;
    if (phi0)
        HIPC(hipMemcpyAsync(h->d_fields, phi0, N * sizeof(double), hipMemcpyHostToDevice, h->s));
    else
        HIPC(launch_phi_builtin(h->d_fields, &h->cfg, h->s));
    HIPC(launch_state_op(h->cfg.precision, 0, h->d_desc, h->d_fields, 0, 0, h->parity, N, h->s));
    // the phase-field-only kernel never writes gbar: keep it zero in both buffers
    if (h->cfg.flow == LB_FLOW_IMPOSED)
        HIPC(launch_state_op(h->cfg.precision, 0, h->d_desc, h->d_fields, 0, 0, h->parity ^ 1, N, h->s));
    HIPC(launch_set_step(h->hdesc.tstep, 0, h->s));
    HIPC(hipStreamSynchronize(h->s));
    h->step = 0;
    h->unstable = false;
    h->diag_pending = false;
    return LB_OK;
}

lb_status lb_set_velocity(lb_handle* h, const double* ux, const double* uy) {
    if (!h || !ux || !uy || h->cfg.flow != LB_FLOW_IMPOSED) return LB_E_INVALID_ARG;
    const int64_t N = (int64_t)h->cfg.nx * h->cfg.ny;
    HIPC(hipMemcpyAsync(h->d_fields, ux, N * sizeof(double), hipMemcpyHostToDevice, h->s));
    HIPC(hipMemcpyAsync(h->d_fields + N, uy, N * sizeof(double), hipMemcpyHostToDevice, h->s));
    HIPC(launch_set_velocity(h->cfg.precision, h->d_desc, h->d_fields, N, h->s));
    HIPC(hipStreamSynchronize(h->s));
    return LB_OK;
}

lb_status lb_step(lb_handle* h, int64_t n) {
    const TraceRange range("lb_step");
    if (!h || n < 0) return LB_E_INVALID_ARG;
    if (h->diag_pending && hipEventQuery(h->ev_diag) == hipSuccess) {
        h->diag_pending = false;
        if (h->h_diag[10] != 0.0) h->unstable = true;
    }
    if (h->unstable) return LB_E_UNSTABLE;
    if (!h->tuned) {
        lb_status st = autotune_single(h);
        if (st != LB_OK) return st;
        h->tuned = true;
    }
    if (h->timing) HIPC(hipEventRecord(h->t0, h->s));
    const int de = h->cfg.diag_every;
    int64_t left = n;
    while (left > 0) {
        int64_t chunk = left;
        if (de > 0) chunk = std::min<int64_t>(left, de - (h->step % de));
        // replay whole graphs where possible, the rest eagerly
        if (chunk >= h->glen) {
            hipGraphExec_t ex;
            const int64_t reps = chunk / h->glen;
            for (int64_t r = 0; r < reps; ++r) {
                lb_status st = graph_for(h, h->parity, &ex);
                if (st != LB_OK) return st;
                HIPC(hipGraphLaunch(ex, h->s));
                h->step += h->glen;
            }
            const lb_status st = launch_steps_eager(h, chunk - reps * h->glen);
            if (st != LB_OK) return st;
        } else {
            const lb_status st = launch_steps_eager(h, chunk);
            if (st != LB_OK) return st;
        }
        left -= chunk;
        if (de > 0 && h->step % de == 0) {
            lb_status st = enqueue_diag(h);
            if (st != LB_OK) return st;
            HIPC(hipMemcpyAsync(h->h_diag, h->d_dout, 16 * sizeof(double), hipMemcpyDeviceToHost, h->s));
            HIPC(hipEventRecord(h->ev_diag, h->s));
            h->diag_pending = true;
        }
    }
    if (h->timing) {
        HIPC(hipEventRecord(h->t1, h->s));
        h->last_steps = n;
    }
    return LB_OK;
}

lb_status lb_get_fields(lb_handle* h, double* phi, double* p, double* ux, double* uy) {
    if (!h) return LB_E_INVALID_ARG;
    const int64_t N = (int64_t)h->cfg.nx * h->cfg.ny;
    HIPC(launch_extract(h->cfg.precision, h->kind, MODE_FIELDS, h->d_desc, h->d_items64, h->n_items64,
                        h->parity, h->s));
    double* outs[4] = {phi, p, ux, uy};
    for (int i = 0; i < 4; ++i)
        if (outs[i])
            HIPC(hipMemcpyAsync(outs[i], h->d_fields + i * N, N * sizeof(double),
                                hipMemcpyDeviceToHost, h->s));
    HIPC(hipStreamSynchronize(h->s));
    return LB_OK;
}

lb_status lb_get_coupling(lb_handle* h, double* dev_out) {
    if (!h || !dev_out) return LB_E_INVALID_ARG;
    LatDesc d = h->hdesc;
    d.fields = dev_out;
    HIPC(hipMemcpyAsync(h->d_desc_cp, &d, sizeof(LatDesc), hipMemcpyHostToDevice, h->s));
    HIPC(launch_extract(h->cfg.precision, h->kind, MODE_COUPLING, h->d_desc_cp, h->d_items64,
                        h->n_items64, h->parity, h->s));
    HIPC(hipStreamSynchronize(h->s));
    return LB_OK;
}

lb_status lb_diagnostics(lb_handle* h, lb_diag* out) {
    if (!h || !out) return LB_E_INVALID_ARG;
    lb_status st = enqueue_diag(h);
    if (st != LB_OK) return st;
    double tmp[16];
    HIPC(hipMemcpyAsync(tmp, h->d_dout, 16 * sizeof(double), hipMemcpyDeviceToHost, h->s));
    HIPC(hipStreamSynchronize(h->s));
    static_assert(sizeof(lb_diag) == 10 * sizeof(double), "lb_diag layout");
    std::memcpy(out, tmp, sizeof(lb_diag));
    return LB_OK;
}

lb_status lb_get_dist(lb_handle* h, double* f, double* g) {
    if (!h) return LB_E_INVALID_ARG;
    const int64_t N = (int64_t)h->cfg.nx * h->cfg.ny;
    double* outs[2] = {f, g};
    if (g && h->cfg.flow == LB_FLOW_IMPOSED) {
        std::memset(g, 0, sizeof(double) * 9 * N);
        outs[1] = nullptr;
    }
    for (int which = 0; which < 2; ++which) {
        if (!outs[which]) continue;
        for (int a = 0; a < 9; ++a) {
            HIPC(launch_state_op(h->cfg.precision, 2, h->d_desc, h->d_fields, a, which, h->parity, N, h->s));
            HIPC(hipMemcpyAsync(outs[which] + a * N, h->d_fields, N * sizeof(double),
                                hipMemcpyDeviceToHost, h->s));
            HIPC(hipStreamSynchronize(h->s));
        }
    }
    return LB_OK;
}

lb_status lb_set_dist(lb_handle* h, const double* f, const double* g, int64_t step) {
    const bool imposed = h && h->cfg.flow == LB_FLOW_IMPOSED;
    if (!h || !f || (!g && !imposed) || step < 0) return LB_E_INVALID_ARG;
    const int64_t N = (int64_t)h->cfg.nx * h->cfg.ny;
    const double* ins[2] = {f, g};
    for (int which = 0; which < (imposed ? 1 : 2); ++which)
        for (int b = 0; b < 9; ++b) {
            HIPC(hipMemcpyAsync(h->d_fields, ins[which] + b * N, N * sizeof(double),
                                hipMemcpyHostToDevice, h->s));
            HIPC(launch_state_op(h->cfg.precision, 1, h->d_desc, h->d_fields, b, which, h->parity, N, h->s));
            HIPC(hipStreamSynchronize(h->s));
        }
    HIPC(launch_set_step(h->hdesc.tstep, (uint32_t)step, h->s));
    HIPC(hipStreamSynchronize(h->s));
    h->step = step;
    h->unstable = false;
    h->diag_pending = false;
    return LB_OK;
}

lb_status lb_state_bytes(lb_handle* h, uint64_t* bytes) {
    if (!h || !bytes) return LB_E_INVALID_ARG;
    *bytes = 16 + (uint64_t)18 * h->plane * h->sbytes;
    return LB_OK;
}

lb_status lb_save_state(lb_handle* h, void* host, uint64_t bytes) {
    if (!h || !host) return LB_E_INVALID_ARG;
    uint64_t need;
    lb_state_bytes(h, &need);
    if (bytes != need) return LB_E_STATE;
    int64_t hdr[2] = {h->step, (int64_t)h->cfg.precision};
    std::memcpy(host, hdr, 16);
    HIPC(hipMemcpyAsync((char*)host + 16, h->buf[h->parity], need - 16, hipMemcpyDeviceToHost, h->s));
    HIPC(hipStreamSynchronize(h->s));
    return LB_OK;
}

lb_status lb_load_state(lb_handle* h, const void* host, uint64_t bytes) {
    if (!h || !host) return LB_E_INVALID_ARG;
    uint64_t need;
    lb_state_bytes(h, &need);
    if (bytes != need) return LB_E_STATE;
    int64_t hdr[2];
    std::memcpy(hdr, host, 16);
    if (hdr[1] != h->cfg.precision || hdr[0] < 0) return LB_E_STATE;
    HIPC(hipMemcpyAsync(h->buf[h->parity], (const char*)host + 16, need - 16, hipMemcpyHostToDevice, h->s));
    HIPC(launch_set_step(h->hdesc.tstep, (uint32_t)hdr[0], h->s));
    HIPC(hipStreamSynchronize(h->s));
    h->step = hdr[0];
    h->unstable = false;
    h->diag_pending = false;
    return LB_OK;
}

lb_status lb_get_step(lb_handle* h, int64_t* step) {
    if (!h || !step) return LB_E_INVALID_ARG;
    *step = h->step;
    return LB_OK;
}

void lb_destroy(lb_handle* h) {
    if (!h) return;
    if (h->s) (void)hipStreamSynchronize(h->s);
    for (int p = 0; p < 2; ++p)
        if (h->gexec[p]) (void)hipGraphExecDestroy(h->gexec[p]);
    if (h->ev_diag) (void)hipEventDestroy(h->ev_diag);
    if (h->t0) (void)hipEventDestroy(h->t0);
    if (h->t1) (void)hipEventDestroy(h->t1);
    if (h->h_diag) (void)hipHostFree(h->h_diag);
    delete h;
}

lb_status lb_timing_enable(lb_handle* h, int32_t on) {
    if (!h) return LB_E_INVALID_ARG;
    h->timing = on != 0;
    h->last_steps = 0;
    return LB_OK;
}

lb_status lb_timing_read(lb_handle* h, double* ms_per_step, int64_t* steps) {
    if (!h || !ms_per_step || !steps) return LB_E_INVALID_ARG;
    *steps = h->last_steps;
    *ms_per_step = 0;
    if (h->last_steps <= 0) return LB_OK;
    HIPC(hipEventSynchronize(h->t1));
    float ms = 0;
    HIPC(hipEventElapsedTime(&ms, h->t0, h->t1));
    *ms_per_step = ms / (double)h->last_steps;
    return LB_OK;
}

lb_status lb_set_schedule(lb_handle* h, int32_t tile_x, int32_t mode, int32_t param, int32_t prefetch) {
    if (!h || mode < 0 || mode > 2 || prefetch < 0 || prefetch > 1) return LB_E_INVALID_ARG;
    if (!valid_width(tile_x, h->cfg.precision, prefetch)) return LB_E_INVALID_ARG;
    if (prefetch && h->kind != KIND_COUPLED_CASCADED) return LB_E_INVALID_ARG;
    if (mode == 0 ? param < kMinH : (param < 1 || param > 4)) return LB_E_INVALID_ARG;
    Sched sc;
    sc.tx = tile_x;
    sc.mode = mode;
    sc.pf = prefetch;
    if (mode == 0) sc.th = param; else sc.mult = param;
    HIPC(hipStreamSynchronize(h->s));
    const lb_status st = set_sched(h, sc);  // LB_E_INVALID_ARG if the cut does not apply
    if (st == LB_OK) h->tuned = true;
    return st;
}

lb_status lb_get_schedule(lb_handle* h, int32_t* tile_x, int32_t* rows, int32_t* grid,
                          int32_t* prefetch) {
    if (!h || !tile_x || !rows || !grid || !prefetch) return LB_E_INVALID_ARG;
    *tile_x = h->sc.tx;
    *rows = h->sc.rows;
    *grid = h->sc.mode != 0 ? h->sc.grid : 0;
    *prefetch = h->sc.pf;
    return LB_OK;
}

lb_status lb_struct_sizes(uint64_t* config_bytes, uint64_t* diag_bytes) {
    if (!config_bytes || !diag_bytes) return LB_E_INVALID_ARG;
    *config_bytes = sizeof(lb_config);
    *diag_bytes = sizeof(lb_diag);
    return LB_OK;
}

lb_status lb_copy_kernel(void* dst, const void* src, uint64_t n, void* stream) {
    if (!dst || !src || ((uintptr_t)dst % 16) || ((uintptr_t)src % 16)) return LB_E_INVALID_ARG;
    HIPC(launch_copy(dst, src, n, (hipStream_t)stream));
    return LB_OK;
}

lb_status lb_bandwidth_probe(void* dst, const void* src, uint64_t n, int32_t variant, void* stream) {
    if (!dst || !src || ((uintptr_t)dst % 16) || ((uintptr_t)src % 16) || variant < 0 || variant > 8)
        return LB_E_INVALID_ARG;
    if (n < ((uint64_t)16 << 20)) return LB_E_INVALID_ARG;  // at least 16 MiB (the read probe's output fits)
    HIPC(launch_bandwidth_probe(dst, src, n, variant, (hipStream_t)stream));
    return LB_OK;
}

}  // extern "C"

// ========================================================================= batch

struct BatchSlot {
    bool used = false;
    lb_config cfg;
    int64_t add_step = 0;  // global step at which the slot was filled
    uint64_t off = 0, bytes = 0;
    int64_t plane = 0;
};

struct lb_batch {
    int prec = 0, nslots = 0, sbytes = 0;
    int kind = -1;  // kernel kind of the occupied slots (-1 while empty)
    int64_t capacity = 0;
    hipStream_t s = nullptr;
    char* ws = nullptr;
    uint64_t ws_bytes = 0;
    LatDesc* d_descs = nullptr;
    std::vector<LatDesc> hdescs;
    WorkItem* d_items = nullptr;
    int max_items = 0, n_items = 0;
    WorkItem* d_items64 = nullptr;
    int max_items64 = 0;
    double* d_fields = nullptr;
    double* d_part = nullptr;
    int max_ny = 0;
    int64_t max_slot_nodes = 0;
    double* d_dout = nullptr;
    char* pool = nullptr;
    uint64_t pool_bytes = 0;
    std::vector<std::pair<uint64_t, uint64_t>> free_list;  // (offset, bytes), sorted
    std::vector<BatchSlot> slot;
    int64_t gstep = 0;
    int parity = 0;
    Sched sc;
    bool fixed_tile = false;
    bool dirty = true;
    bool walls = true;  // some occupied slot has walls (set when the work list is rebuilt)
    bool nt = false;    // every occupied slot's rows are whole cache lines (set with walls)
    int64_t stable = 0;  // steps taken since the work list last changed
    int64_t tuned_nodes = 0;  // nodes in use when the schedule was last autotuned
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int glen = 32;
    int64_t graph_steps = 0;  // steps replayed from captured graphs since creation
    int64_t eager_steps = 0;  // steps launched one by one since creation
    bool timing = false;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    int64_t last_steps = 0;
};

namespace {

// Largest lattice one batch slot may hold (the FP64 read-out scratch is sized for it).
constexpr int64_t kMaxSlotNodes = (int64_t)1 << 24;

struct BatchLayout {
    uint64_t descs, items, items64, part, dout, fields, pool, total;
    int max_items, max_items64, max_ny;
    int64_t max_slot_nodes;
};

BatchLayout batch_layout(int32_t slots, int64_t cap, int prec) {
    BatchLayout L;
    const int sb = store_bytes(prec);
    L.max_items = (int)std::min<int64_t>((int64_t)1 << 30, cap / 32 + 4 * (int64_t)slots + 3 * kMaxGrid);
    L.max_items64 = (int)std::min<int64_t>((int64_t)1 << 30, std::min<int64_t>(cap, kMaxSlotNodes) / 128 + 64);
    L.max_ny = (int)std::min<int64_t>(cap / 8, 1 << 20);
    L.max_slot_nodes = std::min<int64_t>(cap, kMaxSlotNodes);
    uint64_t o = 0;
    L.descs = o; o += align_up((uint64_t)slots * sizeof(LatDesc));
    L.items = o; o += align_up((uint64_t)L.max_items * sizeof(WorkItem));
    L.items64 = o; o += align_up((uint64_t)L.max_items64 * sizeof(WorkItem));
    L.part = o; o += align_up((uint64_t)4 * L.max_ny * sizeof(double));
    L.dout = o; o += align_up(16 * sizeof(double));
    L.fields = o; o += align_up((uint64_t)4 * L.max_slot_nodes * sizeof(double));
    // per slot: two buffers of 18 planes, the per-row table (2 ny doubles <= 2 N bytes)
    // and the step counter
    L.pool = o; o += align_up((uint64_t)2 * 18 * sb * (uint64_t)(cap + 64 * (int64_t)slots) + 2 * (uint64_t)cap +
                              kAlign * 4 * slots);
    L.total = o;
    return L;
}

bool pool_alloc(lb_batch* b, uint64_t bytes, uint64_t* off) {
    bytes = align_up(bytes);
    for (size_t i = 0; i < b->free_list.size(); ++i) {
        auto& fr = b->free_list[i];
        if (fr.second >= bytes) {
            *off = fr.first;
            fr.first += bytes;
            fr.second -= bytes;
            if (fr.second == 0) b->free_list.erase(b->free_list.begin() + i);
            return true;
        }
    }
    return false;
}

void pool_free(lb_batch* b, uint64_t off, uint64_t bytes) {
    bytes = align_up(bytes);
    auto& fl = b->free_list;
    auto it = std::lower_bound(fl.begin(), fl.end(), std::make_pair(off, (uint64_t)0));
    it = fl.insert(it, {off, bytes});
    // coalesce with neighbours
    size_t i = it - fl.begin();
    if (i + 1 < fl.size() && fl[i].first + fl[i].second == fl[i + 1].first) {
        fl[i].second += fl[i + 1].second;
        fl.erase(fl.begin() + i + 1);
    }
    if (i > 0 && fl[i - 1].first + fl[i - 1].second == fl[i].first) {
        fl[i - 1].second += fl[i].second;
        fl.erase(fl.begin() + i);
    }
}

void batch_drop_graphs(lb_batch* b) {
    for (int p = 0; p < 2; ++p)
        if (b->gexec[p]) { (void)hipGraphExecDestroy(b->gexec[p]); b->gexec[p] = nullptr; }
}

std::vector<LatShape> batch_shapes(lb_batch* b) {
    std::vector<LatShape> lats;
    for (int i = 0; i < b->nslots; ++i)
        if (b->slot[i].used) lats.push_back({i, b->slot[i].cfg.nx, b->slot[i].cfg.ny});
    return lats;
}

lb_status batch_set_sched(lb_batch* b, Sched sc) {
    std::vector<WorkItem> items;
    const std::vector<LatShape> lats = batch_shapes(b);
    if (!build_schedule(lats, b->prec, std::max(b->kind, 0), b->walls, sc, b->max_items, items)) {
        // the strip-aligned cut needs lattices of one height: once others have
        // joined, the same grid is cut the general way
        if (sc.mode != 2) return LB_E_WORKSPACE;
        sc.mode = 1;
        if (!build_schedule(lats, b->prec, std::max(b->kind, 0), b->walls, sc, b->max_items, items))
            return LB_E_WORKSPACE;
    }
    if (!items.empty())
        HIPC(hipMemcpyAsync(b->d_items, items.data(), items.size() * sizeof(WorkItem),
                            hipMemcpyHostToDevice, b->s));
    HIPC(hipStreamSynchronize(b->s));
    b->n_items = sc.n_items;
    b->sc = sc;
    batch_drop_graphs(b);
    return LB_OK;
}

lb_status batch_autotune(lb_batch* b) {
    std::vector<LatShape> lats = batch_shapes(b);
    if (lats.empty()) return batch_set_sched(b, b->sc);
    int max_ny = 0;
    std::vector<int> widths;
    for (auto& l : lats) { widths.push_back(l.nx); max_ny = std::max(max_ny, l.ny); }
    // candidate widths are filtered on the median lattice width: narrower lattices
    // then run one strip with idle lanes, which the timing weighs
    std::nth_element(widths.begin(), widths.begin() + widths.size() / 2, widths.end());
    const int med_nx = widths[widths.size() / 2];
    auto timed = [&](Sched& sc, int reps, double* ms) -> lb_status {
        std::vector<WorkItem> items;
        *ms = 1e30;
        if (!build_schedule(lats, b->prec, b->kind, b->walls, sc, b->max_items, items)) return LB_OK;
        HIPC(hipMemcpyAsync(b->d_items, items.data(), items.size() * sizeof(WorkItem),
                            hipMemcpyHostToDevice, b->s));
        *ms = time_candidate(b->prec, b->kind, b->walls, b->nt, sc.tx, sc.pf, b->d_descs, b->d_items, sc.n_items, sc.grid,
                             b->parity, b->s, reps);
        return LB_OK;
    };
    // every candidate once, then the three fastest again with more repetitions
    std::vector<std::pair<double, Sched>> scored;
    for (Sched sc : candidates(b->prec, med_nx, max_ny, b->kind)) {
        double ms;
        const lb_status st = timed(sc, 3, &ms);
        if (st != LB_OK) return st;
        if (ms < 1e30) scored.push_back({ms, sc});
    }
    std::sort(scored.begin(), scored.end(),
              [](const std::pair<double, Sched>& x, const std::pair<double, Sched>& y) { return x.first < y.first; });
    std::vector<std::pair<double, Sched>> fin;
    for (size_t i = 0; i < scored.size() && i < 3; ++i) {
        double ms;
        const lb_status st = timed(scored[i].second, 12, &ms);
        if (st != LB_OK) return st;
        if (ms < 1e30) fin.push_back({ms, scored[i].second});
    }
    return batch_set_sched(b, pick_final(fin, b->sc));
}

lb_status batch_graph(lb_batch* b, int parity, hipGraphExec_t* out) {
    if (!b->gexec[parity]) {
        hipStream_t cs;
        HIPC(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        int p = parity;
        for (int i = 0; i < b->glen && e == hipSuccess; ++i) {
            e = launch_step(b->prec, b->kind, b->walls, b->nt, b->sc.tx, b->sc.pf, b->d_descs, b->d_items, b->n_items, b->sc.grid,
                            p, cs);
            p ^= 1;
        }
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess || e2 != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return LB_E_HIP;
        }
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return LB_E_HIP;
        b->gexec[parity] = ex;
    }
    *out = b->gexec[parity];
    return LB_OK;
}

lb_status batch_extract(lb_batch* b, int32_t slot) {
    const lb_config& c = b->slot[slot].cfg;
    std::vector<WorkItem> it64;
    build_items(slot, c.nx, c.ny, 64, 64, it64);
    if ((int)it64.size() > b->max_items64) return LB_E_WORKSPACE;
    HIPC(hipMemcpyAsync(b->d_items64, it64.data(), it64.size() * sizeof(WorkItem),
                        hipMemcpyHostToDevice, b->s));
    HIPC(launch_extract(b->prec, b->kind, MODE_FIELDS, b->d_descs, b->d_items64, (int)it64.size(), b->parity,
                        b->s));
    return LB_OK;
}

}  // namespace

extern "C" {

lb_status lb_batch_workspace_bytes(int32_t slots, int64_t node_capacity, int32_t precision,
                                   uint64_t* bytes) {
    if (!bytes || slots <= 0 || node_capacity < 64 || store_bytes(precision) == 0) return LB_E_INVALID_ARG;
    *bytes = batch_layout(slots, node_capacity, precision).total;
    return LB_OK;
}

lb_status lb_batch_create(int32_t slots, int64_t node_capacity, int32_t precision, int32_t tile_x,
                          int32_t tile_h, void* dev_ws, uint64_t ws_bytes, void* stream,
                          lb_batch** out) {
    if (!out || !dev_ws || slots <= 0 || node_capacity < 64 || store_bytes(precision) == 0)
        return LB_E_INVALID_ARG;
    if (tile_x != 0 && !valid_width(tile_x, precision, 0)) return LB_E_INVALID_ARG;
    if (tile_h < 0 || (tile_h > 0 && tile_h < kMinH)) return LB_E_INVALID_ARG;
    *out = nullptr;
    const BatchLayout L = batch_layout(slots, node_capacity, precision);
    if (ws_bytes < L.total || ((uintptr_t)dev_ws % kAlign)) return LB_E_WORKSPACE;
    lb_batch* b = new lb_batch();
    b->prec = precision;
    b->nslots = slots;
    b->sbytes = store_bytes(precision);
    b->capacity = node_capacity;
    b->s = (hipStream_t)stream;
    b->ws = (char*)dev_ws;
    b->ws_bytes = ws_bytes;
    b->d_descs = (LatDesc*)(b->ws + L.descs);
    b->hdescs.resize(slots);
    std::memset(b->hdescs.data(), 0, sizeof(LatDesc) * slots);
    b->d_items = (WorkItem*)(b->ws + L.items);
    b->max_items = L.max_items;
    b->d_items64 = (WorkItem*)(b->ws + L.items64);
    b->max_items64 = L.max_items64;
    b->d_part = (double*)(b->ws + L.part);
    b->max_ny = L.max_ny;
    b->max_slot_nodes = L.max_slot_nodes;
    b->d_dout = (double*)(b->ws + L.dout);
    b->d_fields = (double*)(b->ws + L.fields);
    b->pool = b->ws + L.pool;
    b->pool_bytes = L.total - L.pool;
    b->free_list.push_back({0, b->pool_bytes});
    b->slot.resize(slots);
    b->fixed_tile = tile_x != 0 && tile_h != 0;
    b->sc.tx = tile_x ? tile_x : 64;
    b->sc.th = tile_h ? tile_h : 64;
    b->sc.mode = 0;
    if (hipEventCreate(&b->t0) != hipSuccess || hipEventCreate(&b->t1) != hipSuccess) {
        lb_batch_destroy(b);
        return LB_E_HIP;
    }
    *out = b;
    return LB_OK;
}

lb_status lb_batch_add(lb_batch* b, const lb_config* cfg, const double* phi0, int32_t* slot) {
    if (!b || !cfg || !slot || (!phi0 && cfg->init_kind == LB_INIT_NONE)) return LB_E_INVALID_ARG;
    lb_status st = validate(cfg);
    if (st != LB_OK) return st;
    if (cfg->precision != b->prec) return LB_E_INVALID_ARG;
    if (cfg->flow != LB_FLOW_COUPLED) return LB_E_UNSUPPORTED;
    int32_t used_slots;
    int64_t used_nodes;
    lb_batch_usage(b, &used_slots, &used_nodes);
    if (used_slots > 0 && kind_of(cfg) != b->kind) return LB_E_INVALID_ARG;
    if (cfg->ny > b->max_ny || (int64_t)cfg->nx * cfg->ny > b->max_slot_nodes) return LB_E_WORKSPACE;
    int free_slot = -1;
    for (int i = 0; i < b->nslots; ++i)
        if (!b->slot[i].used) { free_slot = i; break; }
    if (free_slot < 0) return LB_E_WORKSPACE;
    const int64_t P = plane_elems(cfg->nx, cfg->ny);
    const uint64_t one = align_up((uint64_t)18 * P * b->sbytes);
    const uint64_t tab = align_up((uint64_t)2 * cfg->ny * sizeof(double));
    const uint64_t ctr = align_up(2 * sizeof(uint32_t));
    uint64_t off;
    if (!pool_alloc(b, 2 * one + tab + ctr, &off)) return LB_E_WORKSPACE;
    BatchSlot& S = b->slot[free_slot];
    S.used = true;
    S.cfg = *cfg;
    S.add_step = b->gstep;
    S.off = off;
    S.bytes = 2 * one + tab + ctr;
    S.plane = P;
    LatDesc& D = b->hdescs[free_slot];
    fill_desc(cfg, D, b->pool + off, b->pool + off + one, P, b->d_fields);
    D.ktab = (double*)(b->pool + off + 2 * one);
    D.tstep = (uint32_t*)(b->pool + off + 2 * one + tab);
    auto undo = [&](lb_status s) {
        S.used = false;
        pool_free(b, off, 2 * one + tab + ctr);
        return s;
    };
    if (hipMemcpyAsync(b->d_descs + free_slot, &D, sizeof(LatDesc), hipMemcpyHostToDevice, b->s) != hipSuccess)
        return undo(LB_E_HIP);
    if (launch_set_step(D.tstep, 0, b->s) != hipSuccess) return undo(LB_E_HIP);
    if (cfg->surf == LB_SIGMA_LANGMUIR && launch_kappa_table(b->d_descs + free_slot, cfg->ny, b->s) != hipSuccess)
        return undo(LB_E_HIP);
    const int64_t N = (int64_t)cfg->nx * cfg->ny;
    if (phi0 ? hipMemcpyAsync(b->d_fields, phi0, N * sizeof(double), hipMemcpyHostToDevice, b->s) != hipSuccess
             : launch_phi_builtin(b->d_fields, cfg, b->s) != hipSuccess)
        return undo(LB_E_HIP);
    // the lattice starts in the buffer the batch's current parity reads
    if (launch_state_op(b->prec, 0, b->d_descs + free_slot, b->d_fields, 0, 0, b->parity, N, b->s) != hipSuccess)
        return undo(LB_E_HIP);
    if (hipStreamSynchronize(b->s) != hipSuccess) return undo(LB_E_HIP);
    if (b->kind != kind_of(cfg)) {  // first lattice of an empty batch sets the kind
        b->kind = kind_of(cfg);
        b->tuned_nodes = 0;
        batch_drop_graphs(b);
    }
    b->dirty = true;
    *slot = free_slot;
    return LB_OK;
}

lb_status lb_batch_remove(lb_batch* b, int32_t slot) {
    if (!b || slot < 0 || slot >= b->nslots || !b->slot[slot].used) return LB_E_INVALID_ARG;
    HIPC(hipStreamSynchronize(b->s));
    pool_free(b, b->slot[slot].off, b->slot[slot].bytes);
    b->slot[slot].used = false;
    b->dirty = true;
    return LB_OK;
}

lb_status lb_batch_step(lb_batch* b, int64_t n, int32_t use_graph) {
    const TraceRange range("lb_batch_step");
    if (!b || n < 0) return LB_E_INVALID_ARG;
    if (b->dirty) {
        int32_t used;
        int64_t nodes;
        lb_batch_usage(b, &used, &nodes);
        // the kernels without wall logic serve batches of periodic lattices only
        b->walls = false;
        b->nt = used > 0 && (uint64_t)2 * 18 * nodes * b->sbytes >= kStreamBytes;
        for (int i = 0; i < b->nslots; ++i) {
            if (!b->slot[i].used) continue;
            if (b->slot[i].cfg.bc_x != LB_PERIODIC || b->slot[i].cfg.bc_y != LB_PERIODIC) b->walls = true;
            if (!b->hdescs[i].ntstore) b->nt = false;
        }
        // autotune when the load changed by more than 2x since the last tuning,
        // otherwise rebuild the work list with the current schedule
        const bool retune = !b->fixed_tile && nodes > 0 &&
                            (b->tuned_nodes == 0 || nodes > 2 * b->tuned_nodes || 2 * nodes < b->tuned_nodes);
        lb_status st = retune ? batch_autotune(b) : batch_set_sched(b, b->sc);
        if (retune && st == LB_OK) b->tuned_nodes = nodes;
        if (st != LB_OK) return st;
        b->dirty = false;
        b->stable = 0;
    }
    if (b->timing) HIPC(hipEventRecord(b->t0, b->s));
    int64_t left = n;
    if (b->n_items > 0) {
        auto eager = [&](int64_t k) -> lb_status {
            for (int64_t i = 0; i < k; ++i) {
                HIPC(launch_step(b->prec, b->kind, b->walls, b->nt, b->sc.tx, b->sc.pf, b->d_descs, b->d_items, b->n_items,
                                 b->sc.grid, b->parity, b->s));
                b->parity ^= 1;
            }
            b->eager_steps += k;
            return LB_OK;
        };
        // graphs only once the work list has held for kGraphAfter graph lengths:
        // while lattices join and leave every few ticks, capturing costs more
        // than it saves.  Within one call, the steps up to that point run one by
        // one and the rest replays graphs.
        if (use_graph) {
            const int64_t gate = (int64_t)kGraphAfter * b->glen;
            const int64_t first = std::min<int64_t>(left, std::max<int64_t>(0, gate - b->stable));
            lb_status st = eager(first);
            if (st != LB_OK) return st;
            left -= first;
            const int64_t reps = left / b->glen;
            for (int64_t r = 0; r < reps; ++r) {
                hipGraphExec_t ex;
                st = batch_graph(b, b->parity, &ex);
                if (st != LB_OK) return st;
                HIPC(hipGraphLaunch(ex, b->s));
            }
            left -= reps * b->glen;  // glen is even: parity unchanged
            b->graph_steps += reps * b->glen;
        }
        const lb_status st = eager(left);
        if (st != LB_OK) return st;
    } else if (n & 1) {
        b->parity ^= 1;
    }
    b->gstep += n;
    b->stable += n;
    if (b->timing) {
        HIPC(hipEventRecord(b->t1, b->s));
        b->last_steps = n;
    }
    return LB_OK;
}

lb_status lb_batch_get_fields(lb_batch* b, int32_t slot, double* phi, double* p, double* ux, double* uy) {
    if (!b || slot < 0 || slot >= b->nslots || !b->slot[slot].used) return LB_E_INVALID_ARG;
    lb_status st = batch_extract(b, slot);
    if (st != LB_OK) return st;
    const int64_t N = (int64_t)b->slot[slot].cfg.nx * b->slot[slot].cfg.ny;
    double* outs[4] = {phi, p, ux, uy};
    for (int i = 0; i < 4; ++i)
        if (outs[i])
            HIPC(hipMemcpyAsync(outs[i], b->d_fields + i * N, N * sizeof(double), hipMemcpyDeviceToHost, b->s));
    HIPC(hipStreamSynchronize(b->s));
    return LB_OK;
}

lb_status lb_batch_diagnostics(lb_batch* b, int32_t slot, lb_diag* out) {
    if (!b || !out || slot < 0 || slot >= b->nslots || !b->slot[slot].used) return LB_E_INVALID_ARG;
    lb_status st = batch_extract(b, slot);
    if (st != LB_OK) return st;
    const lb_config& c = b->slot[slot].cfg;
    const double umax = c.u_max > 0 ? c.u_max : 0.3;
    HIPC(launch_diag(b->d_descs + slot, b->d_fields, b->d_part, b->d_dout, c.ny,
                     (double)(b->gstep - b->slot[slot].add_step), umax, b->s));
    double tmp[16];
    HIPC(hipMemcpyAsync(tmp, b->d_dout, 16 * sizeof(double), hipMemcpyDeviceToHost, b->s));
    HIPC(hipStreamSynchronize(b->s));
    std::memcpy(out, tmp, sizeof(lb_diag));
    return LB_OK;
}

lb_status lb_batch_get_step(lb_batch* b, int32_t slot, int64_t* step) {
    if (!b || !step || slot < 0 || slot >= b->nslots || !b->slot[slot].used) return LB_E_INVALID_ARG;
    *step = b->gstep - b->slot[slot].add_step;
    return LB_OK;
}

lb_status lb_batch_usage(lb_batch* b, int32_t* used_slots, int64_t* used_nodes) {
    if (!b || !used_slots || !used_nodes) return LB_E_INVALID_ARG;
    int32_t u = 0;
    int64_t n = 0;
    for (auto& s : b->slot)
        if (s.used) { ++u; n += (int64_t)s.cfg.nx * s.cfg.ny; }
    *used_slots = u;
    *used_nodes = n;
    return LB_OK;
}

void lb_batch_destroy(lb_batch* b) {
    if (!b) return;
    if (b->s) (void)hipStreamSynchronize(b->s);
    batch_drop_graphs(b);
    if (b->t0) (void)hipEventDestroy(b->t0);
    if (b->t1) (void)hipEventDestroy(b->t1);
    delete b;
}

lb_status lb_batch_timing_enable(lb_batch* b, int32_t on) {
    if (!b) return LB_E_INVALID_ARG;
    b->timing = on != 0;
    b->last_steps = 0;
    return LB_OK;
}

lb_status lb_batch_timing_read(lb_batch* b, double* ms_per_step, int64_t* steps) {
    if (!b || !ms_per_step || !steps) return LB_E_INVALID_ARG;
    *steps = b->last_steps;
    *ms_per_step = 0;
    if (b->last_steps <= 0) return LB_OK;
    HIPC(hipEventSynchronize(b->t1));
    float ms = 0;
    HIPC(hipEventElapsedTime(&ms, b->t0, b->t1));
    *ms_per_step = ms / (double)b->last_steps;
    return LB_OK;
}

lb_status lb_batch_set_schedule(lb_batch* b, int32_t tile_x, int32_t mode, int32_t param, int32_t prefetch) {
    if (!b || mode < 0 || mode > 2 || prefetch < 0 || prefetch > 1) return LB_E_INVALID_ARG;
    if (!valid_width(tile_x, b->prec, prefetch)) return LB_E_INVALID_ARG;
    if (prefetch && b->kind >= 0 && b->kind != KIND_COUPLED_CASCADED) return LB_E_INVALID_ARG;
    if (mode == 0 ? param < kMinH : (param < 1 || param > 4)) return LB_E_INVALID_ARG;
    Sched sc;
    sc.tx = tile_x;
    sc.mode = mode;
    sc.pf = prefetch;
    if (mode == 0) sc.th = param; else sc.mult = param;
    HIPC(hipStreamSynchronize(b->s));
    const Sched old = b->sc;
    const bool old_fixed = b->fixed_tile;
    b->sc = sc;
    b->fixed_tile = true;
    if (!batch_shapes(b).empty()) {  // check that the cut fits now
        const lb_status st = batch_set_sched(b, sc);
        if (st != LB_OK) {
            b->sc = old;
            b->fixed_tile = old_fixed;
            return st == LB_E_WORKSPACE ? LB_E_INVALID_ARG : st;
        }
    }
    b->dirty = true;  // the next step rebuilds the work list with this schedule (and the wall kind)
    return LB_OK;
}

lb_status lb_batch_launch_counts(lb_batch* b, int64_t* graph_steps, int64_t* eager_steps) {
    if (!b || !graph_steps || !eager_steps) return LB_E_INVALID_ARG;
    *graph_steps = b->graph_steps;
    *eager_steps = b->eager_steps;
    return LB_OK;
}

lb_status lb_batch_get_schedule(lb_batch* b, int32_t* tile_x, int32_t* rows, int32_t* grid,
                                int32_t* prefetch) {
    if (!b || !tile_x || !rows || !grid || !prefetch) return LB_E_INVALID_ARG;
    *tile_x = b->sc.tx;
    *rows = b->sc.rows;
    *grid = b->sc.mode != 0 ? b->sc.grid : 0;
    *prefetch = b->sc.pf;
    return LB_OK;
}

}  // extern "C"

// ================================================================ no allocation
//
// lb_step_noalloc advances a lattice whose two state buffers the caller owns,
// with no handle and no workspace.  What the step kernels need beyond those
// buffers -- the lattice descriptor, the step counter that seeds the stochastic
// rounding of 16-bit storage, the work list and (Langmuir law only) the per-row
// kappa~ table -- lives in `scratch`, a file-scope device array of fixed size.
// Each GPU holds its own copy until the process ends; its address on the current
// device is looked up once (hipGetSymbolAddress) and kept per device.  Host code
// uses only that address, never the array's name.  Every call on one device
// rewrites the descriptor, counter, table and work list it uses before its step
// kernels read them, so nothing has to start at zero; calls that overlap on one
// device (different streams, or threads) race on the array.

namespace {

constexpr uint64_t kScratchBytes = (uint64_t)1 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

lb_status scratch_on_current_device(char** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return LB_E_HIP;
    if (dev < 0 || dev >= kMaxDevices) return LB_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LB_E_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = (char*)g_scratch_ptr[dev];
    return LB_OK;
}

// One thread stores the descriptor (passed by value) into device memory.
__global__ void k_put_desc(LatDesc* __restrict__ dst, LatDesc d) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *dst = d;
}

// Work list of one lattice (instance 0), strip-major: item i is row block
// i % nrb of strip i / nrb, th rows of strip_w columns (the host's build_items).
__global__ void k_items_strips(WorkItem* __restrict__ out, int ny, int sw, int th, int nrb, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int st = i / nrb, r = i - st * nrb;
    WorkItem w;
    w.inst = 0;
    w.x0 = st * sw;
    w.y0 = r * th;
    w.y1 = min(ny, r * th + th);
    out[i] = w;
}

}  // namespace

extern "C" {

lb_status lb_step_noalloc(const lb_config* cfg, void* state0, void* state1, uint64_t state_bytes,
                          int64_t step, int64_t n, void* stream) {
    if (!cfg || !state0 || !state1 || n < 0 || step < 0 || state0 == state1) return LB_E_INVALID_ARG;
    lb_status st = validate(cfg);
    if (st != LB_OK) return st;
    if (cfg->flow != LB_FLOW_COUPLED || cfg->diag_every != 0) return LB_E_UNSUPPORTED;
    const int64_t P = plane_elems(cfg->nx, cfg->ny);
    const uint64_t need = (uint64_t)18 * P * store_bytes(cfg->precision);
    if (state_bytes < need || ((uintptr_t)state0 % kAlign) || ((uintptr_t)state1 % kAlign)) return LB_E_WORKSPACE;
    // schedule: one work item per workgroup (the results do not depend on it)
    Sched sc = default_sched(cfg->nx, cfg->ny, kind_of(cfg));
    if (cfg->tile_x) sc.tx = cfg->tile_x;
    if (cfg->tile_h) sc.th = cfg->tile_h;
    if (cfg->tile_x || cfg->tile_h) sc.pf = cfg->tile_pf;
    const int sw = strip_w(sc.tx);
    const int nrb = (cfg->ny + sc.th - 1) / sc.th;
    const int64_t n_items = (int64_t)((cfg->nx + sw - 1) / sw) * nrb;
    // scratch layout: descriptor | step counter | kappa~ table (Langmuir law) | work list
    const uint64_t o_ctr = align_up(sizeof(LatDesc));
    const uint64_t o_tab = o_ctr + align_up(2 * sizeof(uint32_t));
    const uint64_t tab = cfg->surf == LB_SIGMA_LANGMUIR ? align_up((uint64_t)2 * cfg->ny * sizeof(double)) : 0;
    const uint64_t o_items = o_tab + tab;
    if (o_items + (uint64_t)n_items * sizeof(WorkItem) > kScratchBytes) return LB_E_TOO_LARGE;
    if (n == 0) return LB_OK;
    char* scr = nullptr;
    st = scratch_on_current_device(&scr);
    if (st != LB_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    LatDesc D;
    fill_desc(cfg, D, state0, state1, P, nullptr);
    D.ktab = tab ? (double*)(scr + o_tab) : nullptr;
    D.tstep = (uint32_t*)(scr + o_ctr);
    D.vel = nullptr;
    const bool walls = D.wall_y != WALL_NONE || D.wall_x != WALL_NONE;
    LatDesc* d_desc = (LatDesc*)scr;
    WorkItem* d_items = (WorkItem*)(scr + o_items);
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, d_desc, D);
    HIPC(hipGetLastError());
    HIPC(launch_set_step(D.tstep, (uint32_t)step, s));
    hipLaunchKernelGGL(k_items_strips, dim3((unsigned)((n_items + 255) / 256)), dim3(256), 0, s, d_items, cfg->ny,
                       sw, sc.th, nrb, (int)n_items);
    HIPC(hipGetLastError());
    if (tab) HIPC(launch_kappa_table(d_desc, cfg->ny, s));
    const int kind = kind_of(cfg);
    int parity = 0;
    for (int64_t i = 0; i < n; ++i) {
        HIPC(launch_step(cfg->precision, kind, walls, D.ntstore != 0 && 2 * need >= kStreamBytes, sc.tx, sc.pf, d_desc,
                         d_items, (int)n_items, (int)n_items, parity, s));
        parity ^= 1;
    }
    return LB_OK;
}

}  // extern "C"
