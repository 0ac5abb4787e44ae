// Descriptors shared by the host library and the kernels.
#pragma once
#include <stdint.h>

namespace finom {

// One 1D kernel-vector product ("line"): rows xr (R), columns yc (C).
// out_i = log2 sum_j 2^{gin_j - |xr_i - yc_j| kappa} in log2 units
// (kappa = 1/(eps ln 2)), split at the dividing index zeta into the lower
// block (y_j <= x_i) and the upper block (y_j > x_i).
struct LineDesc {
    const double* xr;      // row coordinates, ascending (R)
    const double* yc;      // column coordinates, ascending (C)
    const int* zeta;       // dividing index per row: #{j : yc_j <= xr_i}
    const int* trs;        // merge-path tile row starts (ntiles + 1)
    const double* gin;     // column input, element j at gin[j * gstride]
    double* out;           // row output, element i at out[i * ostride]
    const double* a0;      // epilogue operand, element i at a0[i * ostride]
    const double* a1;      // epilogue operand
    const double* a2;      // epilogue operand
    const void* er;        // fast sweeps: 2^{xr_i kappa} per row (Ext<float>)
    const void* ec;        // fast sweeps: 2^{yc_j kappa} per column (Ext<float>)
    long long R, C;
    long long gstride, ostride;
    double kappa;          // 1 / (eps ln 2)
    double in_scale;       // natural-log input -> log2 units
    double out_scale;      // log2 output -> natural-log output
    double shift;          // coordinate origin used by the moment sums
    int ntiles;
    int agg_base;          // first slot of this line in the tile-aggregate array
    int prob;              // owning problem (state index)
    int part_base;         // partial slot of this line's tile 0 (EPI_UPDATE_CHECK / EPI_COST)
    int dec_part_off;      // first partial slot the stop decision reads (-1: no decision)
    int dec_nparts;        // number of partial slots the stop decision reads
    int writes_state;      // tile 0 of this line records the decision in the state
    int pad;
};

struct WorkItem {
    int line;
    int tile;
};

// Per-problem iteration state, resident on the device. The iteration counter
// is double-buffered by the parity of the graph slot, so the blocks of one
// kernel only read the slot the previous iteration wrote.
struct ProbState {
    int done;              // set once the loop-head check stops the iteration
    int converged;         // err <= tol at the stop
    int status;            // 0 ok, 1 non-finite error
    int pad0;
    long long cnt[2];      // iteration counter, slot = iteration parity
    long long iters;       // completed iterations at the stop
    long long itr_max;
    double err;            // last checked marginal error (L1)
    double tol;
    double w1;             // <C, Gamma> of the returned pair
    double pad1;
};

enum InMode { IN_LOG2 = 0, IN_NAT = 1, IN_LIN = 2 };

enum Epilogue {
    EPI_STORE_LOG2 = 0,    // out = log2 product
    EPI_STORE_NAT = 1,     // out = eps ln product
    EPI_STORE_LIN = 2,     // out = product
    EPI_UPDATE = 3,        // out = a0 - log2 product           (phi = u / K psi)
    EPI_UPDATE_CHECK = 4,  // partial err of |psi_old K^T phi - v|, out = a0 - log2 product
    EPI_COST = 5,          // partial sum of 2^{a0 + log2 moment product}
};

}  // namespace finom
