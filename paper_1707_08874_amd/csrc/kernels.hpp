// Kernel entry points and launch helpers of the HIP library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "consts.hpp"
#include "desc.hpp"
#include "device.hpp"

namespace clsel {

__global__ void k_link_inverse(const double2* links, double2* linv, int64_t links_per_cfg,
                               int nbatch, int32_t* status);
__global__ void k_assemble(const AsmDesc* descs, int ndesc, double2* fronts, int64_t cfg_stride,
                           const int32_t* front_sites, const int32_t* inv_maps,
                           const uint32_t* site_coords, const double2* links, const double2* linv,
                           int64_t link_cfg_stride, const double* mvals, const double* muvals,
                           LatticeDims dims, int32_t* iws, int64_t iws_stride, int fault_cfg,
                           int fault_front);
__global__ void k_gather_zss(const GatherDesc* descs, int ndesc, double2* fronts,
                             int64_t cfg_stride, const int32_t* rel_maps);
__global__ void k_gather_selected(const double2* fronts, int64_t cfg_stride,
                                  const int64_t* sel_off, const int32_t* sel_ld, int64_t V,
                                  int nbatch, const int32_t* status, double2* out);
__global__ void k_drift(const double2* sel, const double2* links, const double2* linv,
                        const double* muvals, LatticeDims dims, int64_t V, int nbatch,
                        double2* out);

__global__ void k_observables(const double2* sel, const double2* links, const double2* linv,
                              const double* muvals, LatticeDims dims, int64_t V, double2* out);

__global__ void k_gauge_drift(const double2* links, const double2* linv, const double* betas,
                              LatticeDims dims, int64_t V, double2* out);
__global__ void k_drift_max(const double2* kf, const double2* kg, int64_t V,
                            unsigned long long* kmax_bits);
__global__ void k_langevin_update(const double2* links_in, double2* links_out, const double2* kf,
                                  const double2* kg, const double* eta, const double* eps_bar,
                                  const double* kref, const unsigned long long* kmax_bits,
                                  int64_t V, double* eps_out);

template <bool TRANS>
__global__ void k_rhs_assemble(const RhsAsmDesc* descs, int ndesc, double2* rhs, int64_t rhs_stride,
                               const double2* b, int64_t b_stride, const int32_t* front_sites,
                               const int32_t* inv_maps, int ns, const int32_t* lim, int64_t lim_stride);
template <bool TRANS>
__global__ void k_rhs_gather(const RhsGatherDesc* descs, int ndesc, double2* rhs, int64_t rhs_stride,
                             const int32_t* rel_maps, int ns, const int32_t* lim, int64_t lim_stride);
template <bool TRANS>
__global__ void k_sol_scatter(const SolScatterDesc* descs, int ndesc, const double2* rhs,
                              int64_t rhs_stride, double2* x, int64_t x_stride,
                              const int32_t* front_sites, int ns, int accumulate, const int32_t* lim,
                              int64_t lim_stride);
__global__ void k_stochastic_blocks(const double2* x, const double2* xi, LatticeDims dims, int64_t V,
                                    int ns, double2* out);

__global__ void k_smw_list(SmwCtx c);
__global__ void k_smw_rhs(SmwCtx c, int which);
__global__ void k_smw_residual(SmwCtx c, const double2* links, const double2* linv, const double* mvals,
                               const double* muvals, LatticeDims dims, int64_t V, int trans);
__global__ void k_smw_residual_delta(SmwCtx c, int trans);
__global__ void k_smw_capacitance(SmwCtx c);
__global__ void k_smw_correct(SmwCtx c, double2* sel, LatticeDims dims, int64_t V);
__global__ void k_smw_gather_rows(SmwCtx c, const double2* x, int64_t x_stride, double2* t,
                                  int64_t t_stride, int ns);

void launch_panel(int rpt, dim3 grid, hipStream_t st, const PanelDesc* descs,
                  const double2* fronts, int64_t cfg_stride, double2* ws, int64_t ws_stride,
                  int32_t* iws, int64_t iws_stride, int32_t* status, double floor);
void launch_gemm(int mode, int tile, dim3 grid, hipStream_t st, const GemmDesc* descs, int ndesc,
                 double2* fronts, int64_t cfg_stride, int64_t pool_elems, double2* ws,
                 int64_t ws_stride, const int32_t* iws, int64_t iws_stride, double2* rhs,
                 int64_t rhs_stride, const int32_t* inv_maps, double2* ext = nullptr,
                 int64_t ext_stride = 0, bool solve = false, const int32_t* lim = nullptr,
                 int64_t lim_stride = 0);

}  // namespace clsel
