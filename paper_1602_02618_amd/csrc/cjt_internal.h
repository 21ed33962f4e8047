// Internal types shared by the HIP sources of libcjt_hip.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

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

// Everything one kernel needs to know about one transform of a launch.  Built
// on the host for every call and copied to the device as an array.
struct ExecDesc {
    int64_t N;          // degree
    int64_t G;          // grid intervals: N (forward) or 2N (inverse)
    double alpha, beta;
    int32_t M;          // Hahn terms
    int32_t nblk;       // Hahn blocks
    int32_t ntasks;     // recurrence tasks
    int32_t pad0;
    int64_t deg_lo[kMaxBlocks], deg_hi[kMaxBlocks];  // half-open degree ranges of the blocks
    int64_t win_lo[kMaxBlocks], win_hi[kMaxBlocks];  // inclusive grid windows of the blocks
    const double* C;          // [M][N+1]   Hahn coefficients C_{n,m}
    const cx<double>* uv;     // [M][G+1]   (u_m, v_m) at the grid points
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
    void* tmp;                // FFT intermediates [nblk*M][L] complex
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

// Wave-uniform copy of an int (the value must already be equal in all lanes).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

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
    // chirp-z only
    int32_t bluestein;
    int32_t logP;
    int64_t P;
    const void* chirp;  // [L]   e^{i pi t^2 / L}
    const void* bl;     // [P]   FFT_P of the kernel conj(chirp) wrapped cyclically
    const void* utw;    // [L+1] e^{i pi s / L}, twiddles of the real-input untangling
};

constexpr int64_t kSingleMax = 4096;
// Largest degree: the inverse's length-2N transform must fit the two-pass
// engine (power-of-two lengths up to 2^22, chirp-z convolutions up to 2^24).
constexpr int64_t kMaxN = (int64_t)1 << 21;

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

// Launchers implemented in the .hip files.
struct EngineArgs {
    const ExecDesc* d_desc;   // device array of descriptors
    int count;                // instances in the launch
    int max_jobs;             // max nblk*M over the instances
    int max_m;                // max M over the instances with blocks
    int max_tasks;            // max ntasks over the instances
    FftGeom geom;             // all instances of one launch share L
    hipStream_t stream;
    // timing labels and algorithmic work of the engine's launches (column pass, row pass)
    const char* name1 = nullptr;
    const char* name2 = nullptr;
    double flops1 = 0, flops2 = 0, bytes1 = 0, bytes2 = 0;
};

enum class Src { FwdAsy, InvAsy, FwdFinal, InvInit, Moments };
enum class Sink { FwdAsy, InvAsy, FwdFinal, InvInit, Weights };

cjt_status launch_rdft(const EngineArgs& a, Src src, Sink sink, bool fp32);
cjt_status launch_rec_fwd(const EngineArgs& a);
cjt_status launch_rec_inv(const EngineArgs& a);
cjt_status launch_rec_inv_reduce(const EngineArgs& a, int64_t maxN);
cjt_status make_twiddles(int64_t L, bool fp32, const void** out, hipStream_t stream);
cjt_status fft_twiddles_cached(int64_t L, bool fp32, hipStream_t st, const void** out);
cjt_status make_chirp_tables(FftGeom* g, bool fp32, hipStream_t st);

}  // namespace cjt
