// Building and running the launch program of a transform call (any mix of
// instances), shared by the one-shot entry points and the persistent batches.
#pragma once

#include <vector>

#include "cjt_internal.h"
#include "plan.h"

// Handle behind cjt_plan_t.
struct cjt_plan_s {
    cjt::Plan p;
};

namespace cjt {

// Where an instance's scratch lives, as byte offsets into the workspace
// (SIZE_MAX: not needed).
struct DescOffsets {
    size_t p, p2, part, tmp, seg;
};

struct Built {
    Program pr;
    std::vector<DescOffsets> offs;
    size_t ws_bytes = 0;      // workspace bytes (persistent part + one chunk of FFT intermediates)
};

// io_off[i]: offset of instance i in the caller's input/output arrays.
// tmp_limit bounds the FFT intermediates held at once (instances are split
// into chunks that run one after the other).  with_patch: the program starts
// with a kernel that sets the in/out pointers from the call's base pointers
// (persistent batches); otherwise the caller sets them before the upload.
cjt_status build_program(const std::vector<const Plan*>& plans, const std::vector<int64_t>& io_off, bool inverse,
                         size_t tmp_limit, bool with_patch, hipStream_t st, Built* out);

// Device pointers of every descriptor from the workspace base.
void bind_workspace(Built& b, void* base);

// Issues the launches: `st` is the caller's stream, `aux` a second stream of
// default priority for the recurrence kernels, fork/join events order them.
cjt_status run_program(const Program& pr, const ExecDesc* d_desc, const Item* d_items, hipStream_t st,
                       hipStream_t aux, hipEvent_t fork, hipEvent_t join, const double* in_base, double* out_base);

}  // namespace cjt
