// Internal declarations of the batched 2D ensemble (host side and kernels).
#pragma once

#include "bbx_internal.h"

namespace bbx {

constexpr int kEnsMaxStim = 8;   // stimuli per tissue
constexpr int kEnsParams = 4;    // model parameters stored per tissue

// One tissue of the ensemble, read by every workgroup of its tiles.
template <typename T>
struct EnsTissue {
    int64_t off;          // first voxel of the tissue in the concatenated arrays
    int nx, ny;
    T cxx, cyy, cxy;      // D_xx/h^2, D_yy/h^2, D_xy/(2h^2)
    T prm[kEnsParams];    // model parameters
    int s0, s1;           // stimuli [s0, s1) of the ensemble's list
};

// A rectangular stimulus; window in whole steps as for a grid.
template <typename T>
struct EnsStim {
    int x0, x1, y0, y1;
    T amp;
    int64_t n0, len, per, count;
};

template <typename T>
struct EnsArgs {
    const int4 *tiles;        // [ntile] (tissue, x0, y0, 0)
    int ntile, per_xcd;
    const EnsTissue<T> *tis;
    const EnsStim<T> *stims;
    T *V0, *V1;               // V ping-pong; step n reads V_{n & 1}
    T *st;                    // [nvar-1][pitch] other state variables
    int64_t pitch;
    T dt;
    double dt64;              // dt in FP64: t_n = n * dt64 for the recorder
    const int64_t *nbase;     // step number of launch j = 0 of this batch
    int rec;
    T theta;
    uint8_t *status;
    T *at, *vmax, *apd, *vrep;
    // 1: state read and V written with non-temporal accesses (ensembles whose state
    // exceeds the Infinity Cache)
    int nt;
};

// Launch step j of a batch (step *nbase + j) with tile variant v.
template <typename T>
hipError_t launch_ens_step(int model, int variant, const EnsArgs<T> &a, int j, hipStream_t s);
// *nbase += k (one thread).
hipError_t launch_ens_advance(int64_t *nbase, int64_t k, hipStream_t s);
// Tile shape (TX, TY) of a variant.
void ens_tile_shape(int variant, int *tx, int *ty);

}  // namespace bbx
