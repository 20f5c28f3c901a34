// Reduced-sweep engine shared by cr_sweep, cr_sweep_batched and the greedy's candidate solves.
#pragma once

#include <vector>

#include "internal.h"

namespace cr {

// One reduced model as seen by the sweep kernel (all pointers device, FP64, column-major).
struct RomDesc {
    const zd* KR;
    const zd* MR;
    const zd* DR;          // may be null (D_R = 0)
    const zd* FR;          // q x L
    const zd* CR;          // n_o x q
    const int32_t* flags;  // L
    const double* omegas;  // frequencies of this model
    zd* out;               // Y: nfreq x L x n_o, or X: nfreq x q x L when out_x
    int q, L, n_o, out_x;
    // frequency-dependent parts: A_R(w_i) += sum_t tcoef[i * nterm + t] T[t]
    int nterm;
    const zd* T[kMaxTerms];
    const zd* tcoef;       // nfreq x nterm (this model's frequencies)
};

struct SweepEngine {
    int num_cu = 256;
    cr_ctx_s* ctx = nullptr;
    DevBuf<RomDesc> d_roms;
    DevBuf<int2> d_items;
    DevBuf<int> d_stats;
    DevBuf<zd> wsA, wsX, wsR, wsB, wsD;
    DevBuf<int> wsP;
    DevBuf<double> d_omega;   // frequencies of the current call
    int qmax = 0, Lmax = 0, nitems = 0;
    // items: (model index, frequency index), processed in the given order by a work queue
    void prepare(const std::vector<RomDesc>& roms, const std::vector<int2>& items, hipStream_t s);
    void launch(cr_precision prec, bool refine, int grid_per_cu, int lds_bytes, hipStream_t s);
    void read_stats(hipStream_t s, int* max_its, int* not_conv, int* perturbed, int* fallbacks);
    void run(const std::vector<RomDesc>& roms, const std::vector<int2>& items, cr_precision prec, bool refine,
             hipStream_t s, int* max_its, int* not_conv, int* perturbed, int grid_override = 0, int* fallbacks = nullptr);
    void autotune(const std::vector<RomDesc>& roms, const std::vector<int2>& items, cr_precision prec, bool refine,
                  hipStream_t s, int* best_gpc, int* best_lds, std::vector<double>* ms);
};

// Allocation-free single-model sweep (cr_sweep_noalloc): every buffer beyond the model, the
// frequencies and Y lives in a static device array. noalloc_scratch_init records that array's
// address on `device` (call with the device current, once per device).
void noalloc_scratch_init(int device);
size_t noalloc_scratch_bytes();
void sweep_noalloc(int device, int num_cu, const RomDesc& rd, const double* omegas_host, int nfreq, cr_precision prec,
                   hipStream_t s, int* max_its, int* not_conv, int* perturbed, int* fallbacks);

}  // namespace cr
