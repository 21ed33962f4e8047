// Plan object and host-side planning helpers.
#pragma once

#include <vector>

#include "cjt_internal.h"

namespace cjt {

// Partition of one grid (Sec. 2.2).  Blocks are rectangles
// [win_lo, win_hi] x [deg_lo, deg_hi) in (grid index, degree).
struct Part {
    int64_t G = 0;        // grid intervals
    int64_t cap = 0;      // highest degree
    int M = 0;            // Hahn terms used
    int64_t n_M = 0;
    double alpha_N = 0.0;
    int K = 0;
    int64_t theta_bar = 0;
    int nblk = 0;
    int exact = 0;        // expansion exact with one term (alpha = beta = 1/2)
    int64_t deg_lo[kMaxBlocks] = {}, deg_hi[kMaxBlocks] = {};
    int64_t win_lo[kMaxBlocks] = {}, win_hi[kMaxBlocks] = {};
    int64_t rec_entries = 0;
};

struct Plan {
    int64_t N = 0;
    double alpha = 0.0, beta = 0.0;
    unsigned flags = 0;
    int device = 0;
    Part fwd, inv;
    std::vector<RecTask> tasks_f, tasks_i;
    int64_t part_total_f = 0, part_total_i = 0;
    // device arena and its views
    void* arena = nullptr;
    size_t arena_bytes = 0;
    double* C = nullptr;
    cx<double>* uv_f = nullptr;
    cx<double>* uv_i = nullptr;
    double* w = nullptr;
    double* s = nullptr;
    d4 *f0 = nullptr, *fp = nullptr, *fm = nullptr;
    d4 *i0 = nullptr, *ip = nullptr, *im = nullptr;
    RecTask* d_tasks_f = nullptr;
    RecTask* d_tasks_i = nullptr;
    bool own_arena = false;      // arena allocated by build_plan_device (else lent by the caller)
    size_t scratch_bytes = 0;    // device scratch build_plan_device needs
    // complex FFT geometries of the two grids, FP64 (geo_*) and in the
    // precision of the Hahn-block FFTs (geob_*); chirp-z tables in the arena
    FftGeom geo_f{}, geo_i{}, geob_f{}, geob_i{};
    // log2 of the column length of the two-pass FFTs of the forward (N) and
    // inverse (2N) grids, from the schedule table at planning time (-1: default)
    int lg1_f = -1, lg1_i = -1;
    // integer parameter shifts (Sec. 1.2): the caller's parameters are
    // (alpha + sh_a, beta + sh_b); alpha, beta above are the core's, in (-1/2, 1/2]
    int sh_a = 0, sh_b = 0;
};

constexpr int kRecWidthFwd = 64 * 4;    // points per forward recurrence task (4 per lane)
constexpr int kRecWidthInv = 64 * 4;    // points per inverse task (4 per lane)

void compute_partition(int64_t G, int64_t cap, double a, double b, int M, Part* P);
void choose_partitions(int64_t N, double a, double b, int M, Part* f, Part* inv);
void build_tasks(const Part& P, int width, std::vector<RecTask>* out, int64_t* part_total);
// Integer shift s and base x - s in (-1/2, 1/2] of a parameter x > -1.
void shift_split(double x, int* shift, double* base);
// Moves the N+1 coefficients v between the caller's parameters and the
// core's (to_base) or back, on st; no-op for plans without shifts.
cjt_status apply_shift(const Plan& P, double* v, bool to_base, hipStream_t st);
// Argument checks shared by every entry point that creates plans.
cjt_status check_args(int64_t N, double alpha, double beta, int M, unsigned flags);
// Host half of plan creation: partitions, recurrence tasks, arena layout.
void plan_host(Plan* P, int64_t N, double alpha, double beta, int M, unsigned flags);
// Sizes of the device arena and of the build scratch (host only; after the
// partitions and tasks are set).
void plan_layout(Plan* P);
// Computes the plan's device arrays on st into `arena` (arena_bytes) using
// `scratch` (scratch_bytes); either may be null, then it is allocated here
// (the arena is then owned by the plan).  Returns after the work completed.
cjt_status build_plan_device(Plan* P, hipStream_t st, void* arena, void* scratch);
// Shape of a length-L complex FFT without tables; lg1 is the log2 column
// length of a two-pass split (-1 or out of range: half the length's bits).
void geometry_shape(int64_t L, FftGeom* g, int lg1);
// Power-of-two length the FFT of length L runs at (L, or P for chirp-z).
int64_t fft_power_length(int64_t L);
// Accepted lg1 range of a two-pass split of a length 2^lg.
void split_range(int lg, int* lo, int* hi);
// Schedule table (csrc/tune.hip): tuned lg1 of the two-pass FFT of power-of-two
// length F for a precision, chirp-z or direct, forward or inverse Hahn blocks;
// -1 when untuned.
int tuned_split(int64_t F, bool fp32, bool chirp, bool inverse);
void set_tuned_split(int64_t F, bool fp32, bool chirp, bool inverse, int lg1);
// Shape plus tables: shared power-of-two twiddles; for lengths that are not
// powers of two, chirp-z tables built into mem (chirp_table_bytes) with
// scratch (chirp_scratch_bytes), asynchronously on st.
cjt_status fft_geometry(int64_t L, bool fp32, hipStream_t st, FftGeom* g, char* mem, char* scratch, int lg1);

}  // namespace cjt
