// Host-callable launchers of the kernels in kernels.hip.  `prec` is
// 0 for FP64 and 1 for FP32-mixed; R is the padded column count of the
// U-like buffers of every instance in the launch.
#pragma once
#include "internal.h"

namespace hl {

enum SpmmModeH : int { SPM_PLAIN = 0, SPM_TRIAL = 1, SPM_AIPP = 2 };
enum RedOpH : int {
  RDH_COMBO = 0, RDH_SDDMM_XT, RDH_TRIAL_PROJ, RDH_PROJ_DOTS, RDH_SDDMM_YP, RDH_AIPP, RDH_EVAL, RDH_LRONLY,
  RDH_LZ_START, RDH_LZ_H1, RDH_LZ_H2, RDH_LZ_FINAL, RDH_FW_DEN, RDH_SETP, RDH_NORM, RDH_GEN_EXTRA, RDH_GRAM,
  RDH_LZ_CHECKH2, RDH_TRIAL_FUSED, RDH_YP_PROJ
};

// coded-diffraction constraints (Section 5.4): per-instance launches around
// the instance's FFTs; total = elements of the launch's index space
void op_cdp_pack(int prec, hipStream_t st, const InstDev *d, int s, int xrole, int vsrc, int R, int Rc,
                 size_t total, int nc);
void op_cdp_abs2(hipStream_t st, const InstDev *d, int s, int Rc, int out, size_t total);
void op_cdp_scale(hipStream_t st, const InstDev *d, int s, int Rc, const double *mult, size_t total);
void op_cdp_gather(hipStream_t st, const InstDev *d, int s, int R, int Rc, int zsel, int vec, size_t total, int nc);
void op_put_params(hipStream_t s, InstParams *dst, const InstParams &v);
// Constraints' low-rank parts: partial K^T X per tile (vsrc 0: role xrole of
// R columns; 1: the Lanczos vector being multiplied; 2: the Ritz vector),
// then per instance the mode's reduction (LcMode).
void op_lc_kty(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int max_rk, int xrole, int vsrc);
void op_lc_sum(hipStream_t s, const int32_t *ilist, int ni, const InstDev *d, int max_rk, int R, int vec);
void op_lc_kz(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int zsel, int vec);
void op_lc_red(hipStream_t s, const int32_t *ilist, int ni, const InstDev *d, int mode, int R, int zsel,
               const double *mult = nullptr);
void op_sddmm(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int xrole, int msel, int wT, int wyp,
              double *tout = nullptr);
void op_lr_dots(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int xrole);
void op_spmm(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int xrole, int msel, int zsel,
             int outrole, int mode);
// rows: total rows of the launch's instances (chooses the grouped or per-tile form)
void op_combo(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int64_t rows);
// SDDMM + gradient SpMM at the trial point in one kernel (narrow rows only)
bool trial_fusable(int prec, int R);
void op_trial_fused(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int xrole);
void op_proj(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int64_t rows);
void op_copy_scale(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int src, int dst);
void op_gram(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, int src);
void op_pack_f64(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, const double *src, int r,
                 int64_t ld, int dst, double scale);
void op_pack_op(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, const void *src, int r,
                int64_t ld, int dst);
void op_unpack_f64(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, double *out, int r,
                   int64_t ld, int src);
void op_unpack_op(int prec, int R, hipStream_t s, const Tile *t, int nt, const InstDev *d, void *out, int r,
                  int64_t ld, int src);
void op_fw_apply(int prec, int RS, int RD, hipStream_t s, const Tile *t, int nt, const InstDev *d, int src, int dst);
void op_rotate(int prec, int RS, int RD, hipStream_t s, const Tile *t, int nt, const InstDev *d, int src, int dst);
void op_gen_constraints(int prec, hipStream_t s, const int32_t *ilist, int ni, int maxm, const InstDev *d, int wT);
void op_pairvals(int prec, hipStream_t s, const int32_t *ilist, int ni, int maxpairs, const InstDev *d, int msel,
                 const double *yext, int general);
void op_fw_den(hipStream_t s, const Tile *t, int nt, const InstDev *d);
void op_fw_den_gen(hipStream_t s, const int32_t *ilist, int ni, int maxm, const InstDev *d);
void op_set_p(hipStream_t s, const int32_t *ilist, int ni, int maxm, const InstDev *d);
void op_refresh_pb(hipStream_t s, const int32_t *ilist, int ni, int64_t maxcount, const InstDev *d);
void op_lower_copy(hipStream_t s, const int32_t *ilist, int ni, int64_t maxnl, const InstDev *d);
void op_reduce(hipStream_t s, const int32_t *ilist, int ni, const InstDev *d, int op, int zsel, int R, int extra);
void op_lz_start(hipStream_t s, const Tile *t, int nt, const InstDev *d);
void op_lz_first(hipStream_t s, const Tile *t, int nt, const InstDev *d);
void op_lz_spmv_dots(hipStream_t s, const Tile *t, int nt, const InstDev *d);
void op_lz_update(hipStream_t s, const Tile *t, int nt, const InstDev *d, int final_pass);
void op_lz_scale(hipStream_t s, const Tile *t, int nt, const InstDev *d);
void op_lz_combine(hipStream_t s, const Tile *t, int nt, const InstDev *d, int to_lzv);

// Allocation-free evaluation (hallar_eval_AUUt_noalloc): the scratch array's
// device address on the current device (resolved once per device), and the
// kernel that copies instance s's descriptor into it with every buffer the
// evaluation writes pointed into the scratch.
hipError_t noalloc_scratch(void **ptr);
void op_noalloc_setup(hipStream_t st, const InstDev *src, int s, const NoallocViews &v);

}  // namespace hl
