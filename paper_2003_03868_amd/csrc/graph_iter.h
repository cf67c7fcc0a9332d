// Device-sized Newton-Schulz iterations replayed from captured hipGraphs
// (graph_iter.hip).
#pragma once

#include "bsm_internal.h"

namespace bsm {

// Device record of one multiply run from the graphs.
struct GiStatus {
    int64_t nnzb_u;      // C blocks before the filter (0 after an overflow)
    int64_t nval_u;      // C scalars before the filter
    int64_t n_groups;    // groups of the group kernel
    int64_t n_entries;   // their entries
    int64_t nnzb;        // C blocks after the filter
    int64_t nval;        // C scalars after the filter
    int64_t n_products;  // block products
    double flops;        // their algorithmic flops, 2 m n k each
    double d;            // square: ||Y - I||_F^2
    int32_t over;        // kGiOver* bits: a fixed-capacity buffer was too small
    int32_t flags;       // kFlagNonFinite from the block products
};
constexpr int kGiOverC = 1, kGiOverG = 2, kGiOverE = 4, kGiOverOut = 8;

struct GraphIter;

// True when X takes the device-sized path: square X with uniform block sizes
// that have an FP64 group kernel, which the multiply would also pick (no
// other kernel variant or tuning-table family asked for), or with sizes in
// {5, 13, 23, 26} when the one-launch paired-group kernel is asked for.
bool graph_iter_ok(const Mat &X);

GraphIter *gi_create(hipStream_t s, double eps, int norm);
void gi_destroy(GraphIter *g);
bool gi_on(const GraphIter *g);
int64_t gi_x_nnzb(const GraphIter *g);

// Take over X (its arrays move into the pools; Y's are released) with
// capacities from the sizes of an eagerly run iteration (square sq, update
// up) times the headroom; (re)allocates and captures the graphs as needed.
int gi_enter(GraphIter *g, Mat &X, Mat &Y, const MulSizes &sq, const MulSizes &up);
// Y = filter(X X) and ||Y - I||_F^2 from the graphs (one wait).
int gi_square(GraphIter *g, GiStatus *out, double *smm_ms);
// X' = filter(1.5 X - 0.5 X Y) from the graphs (one wait); X' becomes X
// unless the record shows an overflow or NaN/Inf.
int gi_update(GraphIter *g, GiStatus *out, double *smm_ms);
// Give X (and Y when y is not NULL) their own arrays again, copied from the
// pools; the pools and graphs stay for a later gi_enter.  If X's copy fails
// (device memory), X keeps no arrays and the iteration stays entered.
int gi_leave(GraphIter *g, Mat &X, Mat *Y);

}  // namespace bsm
