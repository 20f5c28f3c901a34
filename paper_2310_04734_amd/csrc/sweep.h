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
    // Hessenberg-triangular form of the pencil, for models without D_R and terms: Q^H K_R Z = H
    // (upper Hessenberg), Q^H M_R Z = Th (upper triangular), Ft = Q^H F_R, Ct = C_R Z (n_o x q),
    // htnorm = {max |H|, max |Th|}; null when absent
    const zd *H, *Th, *Ft, *Ct;
    const double* htnorm;
};

// One reduction to Hessenberg-triangular form (k_ht_reduce): inputs K_R, M_R, F_R, C_R of one
// model, outputs H, Th, Ft, Ct and htnorm (device, caller-allocated).
struct HtJob {
    const zd *KR, *MR, *FR, *CR;
    zd *H, *Th, *Ft, *Ct;
    double* htnorm;
    int q, L, n_o;
};
constexpr int kHtMaxQ = 512, kHtMaxL = 16, kHtMaxOut = 256;   // limits of the Hessenberg sweep
// whether a model can take the Hessenberg sweep (FP64 sweeps without refinement, outputs Y)
inline bool ht_eligible(int q, int L, int n_o, bool has_d, int nterm) {
    return !has_d && nterm == 0 && q >= 1 && q <= kHtMaxQ && L >= 1 && L <= kHtMaxL && n_o >= 1 && n_o <= kHtMaxOut;
}
void ht_reduce(const std::vector<HtJob>& jobs, hipStream_t s);

struct SweepEngine {
    int num_cu = 256;
    cr_ctx_s* ctx = nullptr;
    DevBuf<RomDesc> d_roms;
    DevBuf<int2> d_items;     // dense-LU items first (nitems), then nht Hessenberg items
    DevBuf<int2> d_redo;      // Hessenberg items handed to the dense path (count in d_stats[6])
    int nht = 0, nht_big = 0, qht = 0;   // Hessenberg items, of which nht_big have q > 256
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
