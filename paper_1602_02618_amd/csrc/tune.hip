// Schedule table of the two-pass FFT splits.  An FFT of power-of-two length
// F = 2^lg above the single-workgroup size runs as column FFTs of length
// 2^lg1 and row FFTs of length 2^(lg - lg1); the split changes the schedule
// (occupancy, transaction sizes, twiddle work), never the arithmetic's
// definition.  cjt_autotune fills the table by timing; plans read it when they
// are made.  The table can be saved and loaded as text, and is loaded once
// from the file named by CJT_TUNE_FILE if that variable is set.
#include <stdio.h>
#include <stdlib.h>

#include <map>
#include <mutex>
#include <tuple>

#include "cjt_internal.h"
#include "plan.h"

namespace cjt {
namespace {

using Key = std::tuple<int64_t, int, int, int>;  // F, fp32, chirp, inverse
std::mutex g_mu;
std::map<Key, int> g_tab;
bool g_env_done = false;

bool valid(int64_t F, int lg1)
{
    if (F <= kSingleMax || (F & (F - 1)) != 0) return false;
    int lg = 0;
    while (((int64_t)1 << lg) < F) ++lg;
    int lo = 0, hi = 0;
    split_range(lg, &lo, &hi);
    return lg1 >= lo && lg1 <= hi;
}

cjt_status load_locked(const char* path)
{
    FILE* f = fopen(path, "r");
    if (!f) return fail(CJT_EINVAL, std::string("cannot read schedule table ") + path);
    std::map<Key, int> tab;
    long long F = 0;
    int inv = 0, chirp = 0, fp32 = 0, lg1 = 0;
    char line[256];
    cjt_status s = CJT_OK;
    while (fgets(line, sizeof(line), f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        if (sscanf(line, "%lld %d %d %d %d", &F, &inv, &chirp, &fp32, &lg1) != 5 || !valid(F, lg1)) {
            s = fail(CJT_EINVAL, std::string("malformed schedule table line: ") + line);
            break;
        }
        tab[Key{F, fp32 != 0, chirp != 0, inv != 0}] = lg1;
    }
    fclose(f);
    if (s == CJT_OK)
        for (auto& e : tab) g_tab[e.first] = e.second;
    return s;
}

void env_locked()
{
    if (g_env_done) return;
    g_env_done = true;
    if (const char* p = getenv("CJT_TUNE_FILE")) (void)load_locked(p);
}

}  // namespace

int tuned_split(int64_t F, bool fp32, bool chirp, bool inverse)
{
    std::lock_guard<std::mutex> lk(g_mu);
    env_locked();
    auto it = g_tab.find(Key{F, fp32, chirp, inverse});
    return it == g_tab.end() ? -1 : it->second;
}

void set_tuned_split(int64_t F, bool fp32, bool chirp, bool inverse, int lg1)
{
    std::lock_guard<std::mutex> lk(g_mu);
    env_locked();
    if (lg1 < 0) g_tab.erase(Key{F, fp32, chirp, inverse});
    else g_tab[Key{F, fp32, chirp, inverse}] = lg1;
}

}  // namespace cjt

using namespace cjt;

extern "C" {

cjt_status cjt_tune_set(int64_t fft_len, int inverse, int chirp, int fp32, int log2_cols)
{
    if (log2_cols >= 0 && !valid(fft_len, log2_cols))
        return fail(CJT_EINVAL, "not a two-pass length or a split outside [max(4, lg-11), min(11, lg-4)]");
    set_tuned_split(fft_len, fp32 != 0, chirp != 0, inverse != 0, log2_cols);
    return CJT_OK;
}

cjt_status cjt_tune_save(const char* path)
{
    if (!path) return fail(CJT_EINVAL, "null path");
    std::lock_guard<std::mutex> lk(g_mu);
    env_locked();
    FILE* f = fopen(path, "w");
    if (!f) return fail(CJT_EINVAL, std::string("cannot write ") + path);
    fprintf(f, "# fft_len inverse chirp fp32 log2_cols\n");
    for (auto& e : g_tab)
        fprintf(f, "%lld %d %d %d %d\n", (long long)std::get<0>(e.first), std::get<3>(e.first), std::get<2>(e.first),
                std::get<1>(e.first), e.second);
    fclose(f);
    return CJT_OK;
}

cjt_status cjt_tune_load(const char* path)
{
    if (!path) return fail(CJT_EINVAL, "null path");
    std::lock_guard<std::mutex> lk(g_mu);
    env_locked();
    return load_locked(path);
}

}  // extern "C"
