// lb_internal.hpp -- declarations shared by the kernels and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cmlb.h"
#include "lb_device.hpp"

namespace cmlb {

// kind: KIND_*; walls false: no lattice of the launch has walls (the kernels
// without wall logic run); nt: every lattice of the launch has rows of whole cache
// lines (LatDesc::ntstore), so widths whose strips are whole lines store
// nontemporally; pf != 0 selects the variant that prefetches the next rows
// (coupled cascaded kind only).
hipError_t launch_step(int prec, int kind, bool walls, bool nt, int tx, int pf, const LatDesc* d,
                       const WorkItem* items, int n_items, int grid, int parity, hipStream_t s);
hipError_t launch_extract(int prec, int kind, int mode, const LatDesc* d, const WorkItem* items64,
                          int n_items, int parity, hipStream_t s);
// stage: FP64 ux plane then uy plane, N values each.
hipError_t launch_set_velocity(int prec, const LatDesc* d, const double* stage, int64_t N, hipStream_t s);
// Per-row Langmuir table of a lattice (d->ktab, 2 ny doubles).
hipError_t launch_kappa_table(const LatDesc* d, int ny, hipStream_t s);
// op 0: init from phi0 plane; 1: set stored plane from staged plane a; 2: get plane a
hipError_t launch_state_op(int prec, int op, const LatDesc* d, double* plane, int a, int which,
                           int cur, int64_t N, hipStream_t s);
hipError_t launch_diag(const LatDesc* d, const double* fields, double* part, double* out, int ny,
                       double step, double u_max, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, uint64_t n, hipStream_t s);
// Sets both slots of a step counter (LatDesc::tstep) to t.
hipError_t launch_set_step(uint32_t* tstep, uint32_t t, hipStream_t s);
// Bandwidth probe variants (see lb_bandwidth_probe in cmlb.h).
hipError_t launch_bandwidth_probe(void* dst, const void* src, uint64_t n, int variant, hipStream_t s);
// Built-in initial phase field of an lb_config (init_kind, init_par, W) into an
// FP64 plane of ny*nx values.
hipError_t launch_phi_builtin(double* out, const lb_config* c, hipStream_t s);
// Resident workgroups per CU of a step kernel (from the HIP occupancy API).
int step_occupancy(int prec, int kind, bool walls, int tx, int pf);

}  // namespace cmlb
