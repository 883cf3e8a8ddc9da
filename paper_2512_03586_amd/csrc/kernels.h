// kernels.h -- argument blocks and host launchers of the engine's kernels.
#pragma once

#include <type_traits>

#include "device.h"

namespace esbgk {

// Arrays of f are of the state's storage type SN (f^n, and f^{n+1} written by
// the final combination) or of the stage arrays' type SS (f^(2), f^(3)); the
// kernels cast them.  The first transported array of an implicit stage is
// f^n, every other transported array is a stage array.  In the mixed form
// (SN = float, SS = bf16_t) the BF16 arrays hold increments: fl[1] of stage 3
// is f^(2) - f^n; stage 3 writes f^(3) (FP32) to fout and P - f^(3) (BF16)
// to sout, and the final combination reads them as fl[0] and fn.
// The implicit term dt A_ij Q'_j of an earlier stage j (at most one: j = 2,
// the array after f^n).  With FP32 or FP64 stage arrays it is taken as
// (A_ij / A_jj)(fq - f*_j), f*_j = f^n - dt ctn L(f^n), ctn = At_j1 (the first
// implicit column is 0); with BF16 stage arrays, whose rounding that
// difference would carry at full weight, as dt A_ij (tau/eps)(Ghat_j - fq)
// with Ghat_j re-evaluated from the per-cell parameters pq stage j wrote.
// 1: FP32 / FP64 stage arrays take the implicit term from the stage
// difference; 0: every form re-evaluates the Gaussian (as the BF16 forms do)
#ifndef ESBGK_QDIFF
#define ESBGK_QDIFF 1
#endif
template <class SS> __host__ __device__ constexpr bool qdiff_form() {
    return ESBGK_QDIFF && !std::is_same<SS, bf16_t>::value;
}

struct StageArgs {
    Geom g;
    const void *fn;                    // f^n: base value at the cell
    const void *fl[2]; double cl[2];   // transport terms  -dt*cl*L(fl)
    const void *fq[1];                 // state of the implicit term
    double qa, qd, qb;                 // A_ij, A_jj, b_j of that term
    double ctn;                        // f*_j = f^n - dt ctn L(f^n)
    const double *pq;                  // Gaussian parameters of stage j (BF16 stage arrays)
    double *pout;                      // Gaussian parameters of this stage (GP_N per cell), or null
    int nl, nq;
    double aii;                        // implicit coefficient; 0 -> final combination
    int emit;                          // write the L1 distance of the result
    void *fout;
    // side output of an implicit stage (state type, at least FP32):
    //   P' = fn - dt sum_l scl[l] L(fl[l]) + dt b_j Q'_j + sfin (fout - f*_i),
    // the last term being dt b_i Q'_i of the stage itself; the final
    // combination reads it as its base
    void *sout; double scl[2]; double sfin;
    double *Uout;                      // SoA [4][nc]
    double *l1out;
    const double *eps;
    const int *list;
    const int *count;
    int *err;
    int nc;
};

template <class S> struct FillArgs {
    Geom g;
    const double *U;
    S *f;
    // mixed form: the BF16 array f^(2) holds f^(2) - f^n; given ref_in (f^n),
    // the fill stores Mhat(U) - ref_in
    const float *ref_in;
    const int *list;
    const int *count;
    int *err;
    int nc;
};

template <class S> struct MomArgs {
    Geom g;
    const S *f;
    double *U;
    double *l1;
    const int *list;
    const int *count;
    int *err;
    int nc;
};

// Euler stage on fluid cells: Uout = Un - dt sum_j cj[j] D_j, D_j the flux
// divergence of state Uj[j].  The divergence of state jnew is formed from its
// stencil (and stored to Dout when given); every other D_j was stored by an
// earlier stage of the step and is read from Dj[j].
struct EulerArgs {
    int nx, ny, nc, recon;
    double dx, dy, dt;
    const double *Un;
    const double *Uj[3];
    const double *Dj[3];
    double cj[3];
    int nj, jnew;
    double *Dout;
    double *Uout;
    const uint8_t *mask;
};

struct IndicatorArgs {
    int nx, ny, nc;
    double twodx, twody;
    double tau, omb;     // omb = 1 - beta
    double cD, ck, cS;
    double eta, delta;
    const double *prim;  // SoA [4][nc] = (rho, ux, uy, T); read when U is null
    const double *U;     // SoA [4][nc] conserved variables: primitives formed in the kernel
    const double *eps;
    const double *l1;
    const uint8_t *mask_old;
    uint8_t *mask_new;
    double *lambda;
};

template <class SN, class SS> hipError_t launch_stage(const StageArgs &a, int nmax, hipStream_t st);
template <class S> hipError_t launch_fill(const FillArgs<S> &a, int nmax, hipStream_t st);
template <class S> hipError_t launch_moments(const MomArgs<S> &a, int nmax, hipStream_t st);
template <class S> hipError_t launch_from_f64(const double *in, void *out, size_t n, hipStream_t st);
template <class S> hipError_t launch_to_f64(const void *in, double *out, size_t n, hipStream_t st);

hipError_t launch_euler(const EulerArgs &a, hipStream_t st);
hipError_t launch_prim(const double *U, double *prim, int nc, hipStream_t st);
hipError_t launch_conserved(const double *rho, const double *ux, const double *uy, const double *T,
                            const double *eps, double *U, double *eps_out, int nc, int *bad,
                            hipStream_t st);
hipError_t launch_indicator(const IndicatorArgs &a, hipStream_t st);
// Classification (1 kinetic, 2 buffer within `radius` cells of a kinetic
// cell, 4 newly kinetic) and the deterministic compaction of the three lists;
// adds the kinetic count to *total when total is given.
hipError_t launch_compact(const uint8_t *mask, const uint8_t *mask_old, uint8_t *cls, int radius, int nx, int ny,
                          int *blockcounts, int *counts, int *kin, int *buf, int *newk, long long *total,
                          hipStream_t st);
hipError_t launch_get_prim(const double *U, double *rho, double *ux, double *uy, double *T, int nc,
                           hipStream_t st);
hipError_t launch_accumulate_count(const int *counts, long long *total, hipStream_t st);
hipError_t launch_zero_fluid_l1(const uint8_t *mask, double *l1, int nc, hipStream_t st);
hipError_t launch_learned_combine(const uint8_t *plain, const float *logits, float threshold, int dilation,
                                  const uint8_t *in_use, uint8_t *out, uint8_t *tmp, int nx, int ny,
                                  long long *counters, hipStream_t st);
}  // namespace esbgk
struct esbgk_mlp;
namespace esbgk {
// Learned-indicator check step: derived fields of the current primitives, then
// mask = plain | (logit > threshold) over the grid; counters (may be null) get
// the judge counts (missed, extra, plain) and one check.
hipError_t launch_learned_mask(esbgk_mlp *m, int nx, int ny, double lx, double ly, const double *prim,
                               const double *eps, const uint8_t *in_use, double *derived, const uint8_t *plain,
                               float threshold, uint8_t *out, long long *counters, hipStream_t st);
int scan_positions(int nx, int ny);
int scan_nblocks(int nx, int ny);

}  // namespace esbgk
