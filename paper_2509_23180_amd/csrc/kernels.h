// Launch wrappers of the HIP kernels (defined in kernels.hip).
#pragma once

#include <vector>

#include <hip/hip_ext.h>

#include "fds_internal.h"


// Kernel launch that carries start/stop events while a timing class is open.
#define FDS_LAUNCH(K, GRID, BLOCK, SMEM, S, ...)                                  \
  do {                                                                          \
    hipEvent_t fds_e0_ = nullptr, fds_e1_ = nullptr;                            \
    if (::fds::Timing::take_pair(&fds_e0_, &fds_e1_))                           \
      hipExtLaunchKernelGGL(K, GRID, BLOCK, SMEM, S, fds_e0_, fds_e1_, 0u, __VA_ARGS__); \
    else                                                                        \
      hipLaunchKernelGGL(K, GRID, BLOCK, SMEM, S, __VA_ARGS__);                 \
  } while (0)

namespace fds {

// Arithmetic / storage combination of a row sine transform:
// D_D: FP64 in, FP64 math, FP64 out;  D_F: FP64 in, FP32 math/out;
// F_F: FP32 throughout;               F_D: FP32 in/math, FP64 out.
enum class DstKind { D_D, D_F, F_F, F_D };

void launch_dst(DstKind kind, const DstTask* tasks, int ntasks, int nblocks, size_t smem, int jidx,
                hipStream_t s);
// Dynamic LDS above 64 KiB must be opted into per kernel (gfx950 has 160 KiB
// per CU).
template <typename K>
inline void ensure_smem(K kernel, size_t smem, size_t* granted) {
  if (smem <= 65536 || smem <= *granted) return;
  if (smem > 160 * 1024) throw Error(FDS_E_UNSUPPORTED, "transform too long for LDS");
  FDS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  *granted = smem;
}

// Wave-parallel variant (one row per 16/32/64 lanes, register budget E).
// Storage types come from DstTask::io_f32 (dst_io_flags(kind)).
inline int dst_io_flags(DstKind k) {
  return ((k == DstKind::F_F || k == DstKind::F_D) ? 1 : 0) |
         ((k == DstKind::D_F || k == DstKind::F_F) ? 2 : 0);
}
void launch_dst_wave(DstKind kind, int E, bool big, const DstTask* tasks, int ntasks, int nblocks,
                     int threads, size_t smem, int jidx, hipStream_t s);
// Matrix-core variant of the row sine transform: RT*16 rows per block, each
// of the 4 waves covers CT*16 columns (4*CT*16 >= n).
size_t gemm_smem_bytes(int n, bool fp32, int rt);
void launch_dst_gemm(DstKind kind, int rt, int ct, const DstTask* tasks, int ntasks, int nblocks,
                     size_t smem, int jidx, hipStream_t s);
void launch_tridiag(bool fp32, const TriTask* tasks, int ntasks, int nblocks, int jidx,
                    hipStream_t s);
// Choice of tridiagonal kernel for a launch whose longest system has
// max_rows rows: the segmented kernel (register segments of `ls` rows, `mpb`
// modes per block, `threads` per block) when the rows fit, else one lane per
// mode sweeping the rows.  FDS_TRI_SEG="mpb,ls" forces a segmented
// configuration (mpb in {8,16,32,64}, ls in {4,8,16}, or 32 for FP32) when
// the rows fit; other values are ignored.
struct TriConfig { bool seg; int ls; int mpb; int threads; };
// The configuration of systems of max_rows rows: FDS_TRI_SEG="mpb,ls" or
// FDS_TRI_TUNE=0 take tri_config_static, otherwise the autotuner's measured
// choice (tune.cpp) among tri_configs(max_rows).
TriConfig tri_config(bool fp32, int max_rows);
TriConfig tri_config_static(bool fp32, int max_rows);
// Every instantiated segmented configuration that holds `rows` rows (the
// unsegmented kernel when none does).
std::vector<TriConfig> tri_configs(int rows);
int tri_blocks(const TriConfig& c, int modes);
void launch_tri(const TriConfig& c, bool fp32, const TriTask* tasks, int ntasks, int nblocks,
                int jidx, hipStream_t s);
// Dense line operators (LineTask::mat): 64 outputs per block, lmax = the
// longest line of the list.
void launch_lines_dense(const LineTask* tasks, int ntasks, int nblocks, int lmax, int jidx,
                        hipStream_t s);
void launch_lines(const LineTask* tasks, int ntasks, size_t smem, int jidx, hipStream_t s);
void launch_operator(int mode, const OpTask* tasks, int ntasks, int nblocks, int jidx,
                     hipStream_t s);
// Dot partials of step j; each problem's last block forms the Gram column and
// the coefficients h_{0..j} (written to KryTask::hv and column j of H).
void launch_gram_dots(const KryTask* tasks, int ntasks, int nblocks, int j, hipStream_t s);
// w - sum h_i v_i into V[j+1]; each problem's last block then takes the norm,
// applies the Givens rotations and tests convergence, and on the end of the
// cycle writes `tag` to flags[KryTask::flag_idx] (flags may be null).
void launch_gram_update(const KryTask* tasks, int ntasks, int nblocks, int j, int* flags, int tag,
                        hipStream_t s);
// Lagged Gram columns (exact preconditioner, restart length m <= kLagMaxJ):
// boundary dots <v_i, s> and the MGS recurrence; the update pass that also
// stores the next Gram column.
void launch_gram_bdots(const KryTask* tasks, int ntasks, int j, hipStream_t s);
void launch_gram_update_lag(const KryTask* tasks, int ntasks, int nblocks, int m, int j, int* flags,
                            int tag, hipStream_t s);
void launch_scale_newest(const KryTask* tasks, int j, int nblocks, hipStream_t s);
void launch_idst_cols(const ColTask* tasks, int ntasks, int nblocks, int jidx, hipStream_t s);
// Hessenberg least squares (back substitution), one workgroup per problem;
// m is the restart length of every task.
void launch_ls_solve(const KryTask* tasks, int ntasks, int m, hipStream_t s);
void launch_combine(bool flex, const KryTask* tasks, int ntasks, int nblocks, hipStream_t s);
void launch_restart(const KryTask* tasks, int ntasks, int nblocks, int initial, int max_cycles,
                    hipStream_t s);
void launch_lift(int mode, const LiftTask* tasks, int ntasks, int nblocks, hipStream_t s);
void launch_iface(const IfaceTask* tasks, int ntasks, hipStream_t s);
void launch_residual(const ResTask* tasks, int ntasks, int nblocks, hipStream_t s);
void launch_res_sum(const ResSumTask* tasks, int ntasks, hipStream_t s);
void launch_copy(const CopyTask* tasks, int ntasks, int nblocks, hipStream_t s);
void launch_count_active(const ProbState* st, int n, int* out, hipStream_t s);

// Interface Krylov iteration (ik_kernels.hip).
void launch_ik_extract(const IkTask* tasks, int ntasks, int nblocks, hipStream_t s);
// max_coords: the largest 1 + nb of the launch's problems
void launch_ik_start(const IkTask* tasks, int ntasks, int max_coords, hipStream_t s);
void launch_ik_cross(const IkTask* tasks, int ntasks, int nblocks, int j, hipStream_t s);
// The two coordinate passes of step j (nblocks: kIkSlab-coordinate blocks).
void launch_ik_wdots(const IkTask* tasks, int ntasks, int nblocks, int j, hipStream_t s);
void launch_ik_update(const IkTask* tasks, int ntasks, int nblocks, int j, int* flags, int tag,
                      hipStream_t s);
void launch_ik_combine(const IkTask* tasks, int ntasks, hipStream_t s);
void launch_ik_compose(const IkTask* tasks, int ntasks, int nblocks, hipStream_t s);
// k_restart alone: the restart decision without scaling a stored V[0].
void launch_restart_decide(const KryTask* tasks, int ntasks, int initial, int max_cycles, hipStream_t s);

// Allocation-free Arnoldi step: size of the per-device scratch array, its
// device address on the current device (looked up once per device), and the
// kernel that clears its partials and writes the state and task records.
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;
void* noalloc_scratch();
void launch_noalloc_setup(double* zero, long long n_zero, ProbState* st, const ProbState& hs,
                          KryTask* dt, const KryTask& t0, const KryTask& t1, hipStream_t s);

}  // namespace fds
