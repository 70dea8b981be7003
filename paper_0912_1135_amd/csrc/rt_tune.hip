// Autotuner of the preconditioner's large contractions.  For a shape not
// seen before, every candidate configuration runs once on the plan's stream
// with the plan's real operands, timed with HIP events; the fastest is kept
// in a process-wide table keyed by the operation and its sizes, used by every
// later preconditioning of that shape, and can be saved to and loaded from a
// text file (one "key choice..." line per entry).
#include "rt_plan_state.h"

#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

namespace {

std::mutex g_tune_mutex;
std::map<std::string, std::vector<int>> g_tune;

}  // namespace

namespace rtp {

std::string tune_key(const char *op, int64_t m, int64_t n, int64_t k)
{
    std::ostringstream os;
    os << op << ':' << m << 'x' << n << 'x' << k;
    return os.str();
}

bool tune_lookup(const std::string &key, std::vector<int> &choice)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    choice = it->second;
    return true;
}

void tune_store(const std::string &key, const std::vector<int> &choice)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune[key] = choice;
}

rtproj_status tune_pick(rtproj_plan p, int count, const std::function<hipError_t(int)> &run, int *best,
                        std::vector<float> *times)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    RT_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(RTPROJ_ERR_DEVICE, "hipEventCreate failed");
    }
    float best_ms = INFINITY;
    *best = 0;
    hipError_t err = hipSuccess;
    for (int c = 0; c < count && err == hipSuccess; ++c) {
        (void)hipEventRecord(e0, p->stream);
        err = run(c);
        (void)hipEventRecord(e1, p->stream);
        if (err != hipSuccess) break;
        (void)hipEventSynchronize(e1);
        float ms = INFINITY;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (times) times->push_back(ms);
        if (ms < best_ms) { best_ms = ms; *best = c; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    RT_HIP(err);
    return RTPROJ_OK;
}

}  // namespace rtp

using namespace rtp;

extern "C" {

rtproj_status rtproj_plan_set_autotune(rtproj_plan p, int enable)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    p->autotune = enable != 0;
    return RTPROJ_OK;
}

rtproj_status rtproj_autotune_save(const char *path)
{
    if (!path) return fail(RTPROJ_ERR_INVALID_ARG, "path is NULL");
    std::ofstream f(path);
    if (!f) return fail(RTPROJ_ERR_INVALID_ARG, std::string("cannot write ") + path);
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    for (const auto &kv : g_tune) {
        f << kv.first;
        for (int v : kv.second) f << ' ' << v;
        f << '\n';
    }
    return f ? RTPROJ_OK : fail(RTPROJ_ERR_INVALID_ARG, std::string("write failed: ") + path);
}

rtproj_status rtproj_autotune_load(const char *path)
{
    if (!path) return fail(RTPROJ_ERR_INVALID_ARG, "path is NULL");
    std::ifstream f(path);
    if (!f) return fail(RTPROJ_ERR_INVALID_ARG, std::string("cannot read ") + path);
    std::string line;
    std::map<std::string, std::vector<int>> got;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string key;
        if (!(is >> key)) continue;
        std::vector<int> v;
        int x;
        while (is >> x) v.push_back(x);
        if (v.empty() || key.find(':') == std::string::npos)
            return fail(RTPROJ_ERR_INVALID_ARG, "malformed tuning line: " + line);
        got[key] = v;
    }
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    for (auto &kv : got) g_tune[kv.first] = kv.second;
    return RTPROJ_OK;
}

int rtproj_autotune_entries(void)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    return (int)g_tune.size();
}

}  // extern "C"
