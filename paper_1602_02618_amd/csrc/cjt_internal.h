// Internal types shared by the HIP sources of libcjt_hip.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/cjt.h"

namespace cjt {

constexpr int kMaxBlocks = CJT_MAX_BLOCKS;
constexpr int kMaxM = 30;

// Complex value in registers / LDS / global memory.
template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T re, im;
};

// Four coefficients of one degree of a recurrence, loaded as one record.
struct alignas(32) d4 {
    double x, y, z, w;
};

// A group of grid points handled by one recurrence work-item: points
// p0 .. p0+np-1, all with the same recurrence form (mode 0 = three-term
// recurrence, +1 / -1 = the modified form anchored at x0 = +1 / -1) and the same
// number of degrees `cut` left to recurrence.  `off` is the offset of this
// task's partial sums (inverse direction only).
struct RecTask {
    int32_t p0;
    int32_t np;
    int32_t mode;
    int32_t cut;
    int64_t off;
};

// Geometry of one complex FFT length L on the device.  Powers of two run
// directly; any other L runs as a cyclic convolution of power-of-two length
// P >= 2L-1 (Bluestein's chirp-z identity), with the same radix kernels.
struct FftGeom {
    int64_t L;        // complex length
    int32_t logL;
    int32_t single;   // 1: whole transform in one workgroup
    int32_t L1, L2;   // two-pass split of the power-of-two length (L, or P for chirp-z)
    int32_t logL1, logL2;
    const void* tw;   // [2L'] e^{i pi q / L'}, L' = L (power of two) or P (chirp-z)
    const void* tw1;  // [2 L1] e^{i pi q / L1}: stages of the column FFTs (two passes only)
    const void* tw2;  // [2 L2] e^{i pi q / L2}: stages of the row FFTs
    // chirp-z only
    int32_t bluestein;
    int32_t logP;
    int64_t P;
    const void* chirp;  // [L]   e^{i pi t^2 / L}
    const void* bl;     // [P]   FFT_P of the kernel conj(chirp) wrapped cyclically: natural order
                        //       (one workgroup), row-major [k1][k2] for frequency k1 + L1 k2 (two passes)
    const void* utw;    // [L+1] e^{i pi s / L}, twiddles of the real-input untangling
};

// Everything one kernel needs to know about one transform of a launch.  Built
// on the host for every call and copied to the device as an array.
struct ExecDesc {
    int64_t N;          // degree
    int64_t G;          // grid intervals: N (forward) or 2N (inverse)
    double alpha, beta;
    int32_t M;          // Hahn terms
    int32_t nblk;       // Hahn blocks
    int32_t ntasks;     // recurrence tasks
    int32_t rec_seg;    // recurrence segment length: tasks with more than 2 rec_seg degrees are split
    int64_t deg_lo[kMaxBlocks], deg_hi[kMaxBlocks];  // half-open degree ranges of the blocks
    int64_t win_lo[kMaxBlocks], win_hi[kMaxBlocks];  // inclusive grid windows of the blocks
    const double* C;          // [M][N+1]   Hahn coefficients C_{n,m}
    const cx<double>* uv;     // [M][G+1]   (u_m, v_m) at the grid points; inverse: planes (u_m+v_m)/2, (u_m-v_m)/2
    const double* w;          // [2N+1]     Clenshaw--Curtis weights (inverse)
    const double* s;          // [N+1]      1 / A_n (inverse)
    const RecTask* tasks;     // [ntasks]   recurrence tasks, longest first
    const d4* rec0;      // [N+2]      three-term coefficients
    const d4* recp;      // [N+2]      modified form at x0 = +1
    const d4* recm;      // [N+2]      modified form at x0 = -1
    const double* in;         // input coefficients (N+1)
    double* out;              // output coefficients (N+1)
    double* p;                // forward: recurrence part of the point values (N+1); inverse: g = w .* f (2N+1)
    double* p2;               // forward: Hahn-block part of the point values (N+1)
    double* part;             // inverse: recurrence partial sums
    void* tmp;                // FFT intermediates, fft_job_bytes(L) per job
    double* seg;              // recurrence segment records (long recurrences split in degree)
    int64_t io_off;           // offset of this instance in the caller's input / output arrays
    FftGeom geo;              // FFT of length L = G (FP64 tables)
    FftGeom geob;             // the same length in the precision of the Hahn-block FFTs
};

// One work item of a launch: which descriptor it serves and up to three
// kernel-specific indices (job, tile, task, segment, record slot, ...).
struct Item {
    int32_t desc, a, b, c;
};

// Read-only views in the constant address space: loads from wave-uniform
// addresses through these become scalar (s_load) instructions.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p)
{
    return (cptr<T>)p;
}

// Loads through the constant address space, member by member (C++ copies do
// not bind to address-space-qualified references).
__device__ __forceinline__ d4 ld(cptr<d4> p) { return d4{p->x, p->y, p->z, p->w}; }

// Global-memory accessors.  The device pointers of a descriptor are read
// from memory, so the compiler cannot tell that they point to global memory
// and would use flat instructions: 64-bit per-lane addresses, and a shared
// wait counter with LDS, so every LDS wait would also wait for the loads in
// flight.  Going through address space 1 gives global loads/stores with a
// scalar base and a 32-bit lane offset.
template <typename T>
using gptr = T __attribute__((address_space(1)))*;

template <typename T>
struct vec2_of;
template <>
struct vec2_of<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct vec2_of<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};
// two consecutive doubles at an address that is only 8-byte aligned
typedef double dpair8 __attribute__((ext_vector_type(2), aligned(8)));

__device__ __forceinline__ double ldg(const double* p) { return *(gptr<const double>)p; }
__device__ __forceinline__ float ldg(const float* p) { return *(gptr<const float>)p; }
__device__ __forceinline__ int32_t ldg(const int32_t* p) { return *(gptr<const int32_t>)p; }
__device__ __forceinline__ int64_t ldg(const int64_t* p) { return *(gptr<const int64_t>)p; }
__device__ __forceinline__ void stg(double* p, double v) { *(gptr<double>)p = v; }
template <typename T>
__device__ __forceinline__ cx<T> ldg(const cx<T>* p)
{
    typedef typename vec2_of<T>::type V;
    const V v = *(gptr<const V>)p;
    return {v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void stg(cx<T>* p, cx<T> a)
{
    typedef typename vec2_of<T>::type V;
    V v;
    v.x = a.re;
    v.y = a.im;
    *(gptr<V>)p = v;
}
__device__ __forceinline__ dpair8 ldg_pair(const double* p) { return *(gptr<const dpair8>)p; }
// one recurrence coefficient record (32 bytes, 32-byte aligned)
__device__ __forceinline__ d4 ldg(const d4* p)
{
    typedef double V __attribute__((ext_vector_type(4)));
    const V v = *(gptr<const V>)p;
    return d4{v.x, v.y, v.z, v.w};
}

// Wave-uniform copy of an int (the value must already be equal in all lanes).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Workgroup b of a launch runs on XCD b mod 8 (each XCD has its own L2).
// Launches whose neighbouring items share inputs map workgroups to items so
// that every XCD takes one contiguous range of the item list.
__device__ __forceinline__ int64_t xcd_item(int64_t b, int64_t nb)
{
    constexpr int64_t X = 8;
    const int64_t q = nb / X, r = nb % X, x = b % X, i = b / X;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

constexpr int64_t kSingleMax = 4096;
// Largest degree: the inverse's length-2N transform must fit the two-pass
// engine (power-of-two lengths up to 2^22, chirp-z convolutions up to 2^24).
constexpr int64_t kMaxN = (int64_t)1 << 21;
constexpr double kMaxShiftParam = 2.5;  // CJT_SHIFT: at most 2 unit shifts up per parameter

// Bytes of intermediate storage one job of the FFT engine needs for length L.
size_t fft_job_bytes(int64_t L, bool fp32);

// Error reporting (thread-local detail message).
void set_error(const std::string& msg);
cjt_status fail(cjt_status st, const std::string& msg);

#define CJT_HIP_TRY(expr)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::cjt::fail(CJT_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Kernel timing (see cjt_profile_enable): brackets one launch with HIP events
// on `stream` when timing is on, tagged with the launch's algorithmic work.
struct ProfScope {
    ProfScope(const char* name, double flops, double bytes, hipStream_t stream);
    ~ProfScope();
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;
    bool on = false;
    int slot = -1;
    hipStream_t st = nullptr;
};

enum class Src { FwdAsy, InvAsy, FwdFinal, InvInit, Moments };
enum class Sink { FwdAsy, InvAsy, FwdFinal, InvInit, Weights };

// Kernels of the engine.  A transform call is a list of launches, each over a
// flat list of work items that may mix instances of any degree.
enum class Kind : int32_t {
    Fork,            // the auxiliary stream waits for the caller's stream
    Join,            // the caller's stream waits for the auxiliary stream
    Patch,           // in/out pointers of every descriptor from the call's base pointers
    FftSingle,       // whole power-of-two transform in one workgroup, all jobs of an instance
    FftPass1,        // column pass of a two-pass transform, one (job, column tile)
    FftPass1Terms,   // Hahn blocks: column pass of every block of one (term, column tile)
    FftPass2,        // row pass + untangling + sink, all jobs (or one job) of an instance, one row tile
    JobRowReduce,    // sum of the per-job row-pass parts in job order, then the sink
    BsSingle,        // chirp-z transform in one workgroup
    BsCol1,     // chirp-z, two passes: column pass of the first transform
    BsRowConv,  // row FFT, kernel product, inverse row FFT, in place
    BsCol2Inv,  // inverse column FFT, chirp, to Z
    BsUntangle,      // chirp-z untangling + sink
    FftJobs,         // one job of a power-of-two single-workgroup transform, sink parts per job
    BsJobs,          // one job of a chirp-z single-workgroup transform, sink parts per job
    JobReduce,       // sum of the per-job sink parts
    RecFwd,          // forward recurrence over the whole degree range of a task
    RecFwdSeg,       // forward recurrence over one degree segment of a long task (affine map)
    RecFwdCombine,   // forward: chain the affine maps of a split task's segments
    RecInvMaps,      // inverse: transfer maps of a split task's segments
    RecInvInit,      // inverse: starting state of every segment of a split task
    RecInv,          // inverse recurrence over a degree segment, reduced over points
    RecInvReduce,    // inverse: sum of task partials, Hahn part, 1/A_n
};

struct Launch {
    Kind kind;
    int32_t stream = 0;        // 0: the caller's stream, 1: the auxiliary stream
    Src src = Src::FwdAsy;
    Sink sink = Sink::FwdAsy;
    int32_t fp32 = 0;          // FFT arithmetic in FP32
    int32_t nth = 0;           // threads per workgroup
    int64_t item_off = 0;      // first item in the program's item array
    int64_t nitems = 0;
    size_t lds = 0;            // dynamic LDS bytes
    size_t acc_off = 0;        // kernel-specific LDS offset
    int32_t seg = 0;           // recurrence segment length (degrees)
    const char* name = nullptr;
    double flops = 0, bytes = 0;
};

struct Program {
    std::vector<ExecDesc> descs;
    std::vector<Item> items;
    std::vector<Launch> launches;
};

// Appends the launches of one pass of the FFT engine over the instances
// `which` (indices into pr.descs).  flops/bytes: algorithmic work per
// instance, for the timing labels.
cjt_status add_fft(Program& pr, const std::vector<int>& which, Src src, Sink sink, bool fp32, int stream,
                   const char* name_cols, const char* name_rows, const std::vector<double>& flops,
                   const std::vector<double>& bytes, bool job_parallel = false);
// Intermediate bytes one instance needs for a pass of `jobs` jobs over the
// length of geometry g (0: none), in the mode add_fft will choose.
size_t fft_tmp_bytes(const FftGeom& g, int64_t jobs, bool fp32, bool job_parallel);
// Recurrence launches over all instances.  Each descriptor's rec_seg splits
// its tasks longer than 2 rec_seg degrees.  rec_segment_length picks it from
// the total work of `which` instances (all of them: the whole call; one: an
// instance alone, for results that do not depend on the rest of the call);
// rec_seg_doubles gives the segment-record doubles an instance then needs.
int32_t rec_segment_length(const Program& pr, const std::vector<const RecTask*>& tasks, const std::vector<int>& which);
int64_t rec_seg_doubles(const ExecDesc& d, const RecTask* tasks);
void add_rec_fwd(Program& pr, const std::vector<const RecTask*>& tasks, int stream, double flops, double bytes);
void add_rec_inv(Program& pr, const std::vector<const RecTask*>& tasks, int stream, double flops, double bytes);
void add_rec_inv_reduce(Program& pr, int stream, double bytes);

cjt_status launch_fft(const Launch& L, const ExecDesc* d_desc, const Item* d_items, hipStream_t s);
cjt_status launch_rec(const Launch& L, const ExecDesc* d_desc, const Item* d_items, hipStream_t s);
cjt_status make_twiddles(int64_t L, bool fp32, const void** out, hipStream_t stream);
cjt_status fft_twiddles_cached(int64_t L, bool fp32, hipStream_t st, const void** out);
// Chirp-z tables of a non-power-of-two geometry: device bytes they occupy,
// scratch bytes their construction needs, and the construction itself into
// caller memory (owned by the plan of that length).
size_t chirp_table_bytes(const FftGeom& g, bool fp32);
size_t chirp_scratch_bytes(const FftGeom& g, bool fp32);
cjt_status make_chirp_tables(FftGeom* g, bool fp32, hipStream_t st, char* mem, char* scratch);

}  // namespace cjt
