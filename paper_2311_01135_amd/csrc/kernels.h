// Host-side launchers of the HIP kernels (one translation unit per family).
#pragma once

#include "ks_internal.h"

namespace ks {

// error plumbing
void set_error(const char* fmt, ...);
#define KS_HIP(x)                                                                  \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            ks::set_error("%s failed: %s (%s:%d)", #x, hipGetErrorString(e_),     \
                          __FILE__, __LINE__);                                     \
            return KS_EDEVICE;                                                     \
        }                                                                          \
    } while (0)

// timing of kernel families (no-op unless b->timing)
struct KTimer {
    ks_batch* b;
    const char* name;
    hipStream_t s;
    hipEvent_t e0{}, e1{};
    KTimer(ks_batch* b_, const char* n, hipStream_t s_);
    KTimer(ks_batch* b_, const char* n) : KTimer(b_, n, b_->stream) {}
    ~KTimer();
};
// Makes the batch stream wait for a grid still being built on the aux stream.
ks_status grid_wait(ks_batch* b);
void resolve_timers(ks_batch* b);

// integrals (k_ints.hip)
void build_boys_table(std::vector<double>& tab);
void build_boys_rows(std::vector<double>& rows);
ks_status launch_int1e(ks_batch* b);
ks_status launch_pairs(ks_batch* b);
ks_status launch_eri(ks_batch* b);
ks_status launch_eri_unpack(const ks_batch* b, int mol, double* d_out);
ks_status launch_eri_unpack_window(const ks_batch* b, int mol, long lo, long hi, double* d_out);
// Schwarz factors Q_ab = max_component sqrt|(ab|ab)| of every shell pair.
ks_status launch_schwarz(ks_batch* b);
ks_status sort_pairs_by_schwarz(ks_batch* b);
ks_status launch_permute_pairs(ks_batch* b, int c, const int* perm, Pair* pairs_out, int2* pao_out, double* pp_out,
                               double* Q_out);
// Integral-direct J/K: the ERIs of every quartet that survives the
// density-weighted Schwarz test are computed and digested on the fly.
ks_status launch_direct_jk(ks_batch* b, const double* P, double* J, double* K, bool only_active, bool incremental,
                           bool track);

// J/K (k_jk.hip)
// incremental: digest P - Pprev and add to J, K; track: afterwards Pprev = P.
ks_status launch_jk(ks_batch* b, const double* P, double* J, double* K, bool only_active, bool incremental,
                    bool track);
size_t jk_lds_bytes(const ks_batch* b);
// J = sum_chunks (AJ + AJ^T), K likewise, from the per-work-item partials.
ks_status launch_jk_reduce(ks_batch* b, bool acc_fp64, const double* P, double* J, double* K, bool only_active,
                           bool incremental, bool track);
bool jk_acc_fp64(const ks_batch* b);
int jk_mode(const ks_batch* b);     // 0 LDS FP64, 1 LDS FP32, 2 global FP64 accumulation
// dP = P - Pref (or P) into the batch work area, for global-mode digestion
ks_status launch_delta(ks_batch* b, const double* P, const double* Pref, bool only_active);

// grid and XC (k_xc.hip)
ks_status launch_grid(ks_batch* b, hipStream_t s);
ks_status launch_xc(ks_batch* b, const double* P, double* V, bool only_active);
size_t xc_lds_bytes(const ks_batch* b);
int xc_block_points(const ks_batch* b);
struct XcShape { int bp = 32, nw = 8; bool pglobal = false; size_t lds = 0; };
XcShape xc_shape(const ks_batch* b);

// SCF steps (k_scf.hip)
ks_status launch_fock(ks_batch* b, const double* P, const double* J, const double* K, const double* Vxc,
                      double* F, bool only_active, double* d_eterms);
ks_status launch_lowdin(ks_batch* b);
ks_status launch_guess(ks_batch* b);
ks_status launch_iteration_tail(ks_batch* b);
ks_status launch_count_active(ks_batch* b);

// SCF driver pieces (abi.hip) used by the server
ks_status step_launch(ks_batch* b);
ks_status step_finish(ks_batch* b, int* n_active);
size_t batch_device_bytes(const ks_batch* b);

}  // namespace ks
