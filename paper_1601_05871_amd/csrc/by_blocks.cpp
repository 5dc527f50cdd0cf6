// flame_factor_by_blocks: Cholesky-by-blocks on a device task DAG (k_dag.hip)
// for a dense matrix or a block pattern.  The task list of a (block count,
// pattern) pair is built once on the host and kept; it is copied into the
// library workspace whenever that workspace has been replaced or last held
// another list.
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "flame_internal.h"

namespace flame {
std::vector<int4> by_blocks_tasks(int nbt, const uint8_t *pattern);
int launch_by_blocks(int64_t n, double *A, int64_t lda, const int4 *tasks, int64_t ntasks, int nbt, int32_t *ints,
                     int32_t *info, hipStream_t s);
}  // namespace flame

using namespace flame;

namespace {

constexpr int64_t kBlock = 128;

struct DagEntry {
    std::vector<int4> tasks;
};
std::mutex g_dag_mu;
std::map<std::pair<int, std::vector<uint8_t>>, DagEntry> g_dag_lists;
// what the workspace of each device holds: (its generation, the list's key)
std::map<int, std::pair<uint64_t, const DagEntry *>> g_dag_uploaded;

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

namespace flame {

int by_blocks_factor(int64_t n, double *A, int64_t lda, const uint8_t *pattern, int32_t *info, hipStream_t s) {
    const int nbt = (int)((n + kBlock - 1) / kBlock);
    std::vector<uint8_t> pat;
    if (pattern != nullptr && nbt > 0) {
        // the upper triangle of the pattern (diagonal blocks always exist)
        pat.assign((size_t)nbt * nbt, 0);
        for (int i = 0; i < nbt; ++i)
            for (int j = i; j < nbt; ++j) pat[(size_t)i * nbt + j] = (i == j || pattern[(size_t)i * nbt + j]) ? 1 : 0;
    }
    DevCtx *ctx = ctx_for_current_device();
    if (ctx == nullptr) return FLAME_ERR_HIP;
    int dev = 0;
    FLAME_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_dag_mu);
    auto key = std::make_pair(nbt, pat);
    auto it = g_dag_lists.find(key);
    if (it == g_dag_lists.end())
        it = g_dag_lists.emplace(key, DagEntry{by_blocks_tasks(nbt, pat.empty() ? nullptr : pat.data())}).first;
    const DagEntry *e = &it->second;
    const size_t task_bytes = up256(e->tasks.size() * sizeof(int4));
    const size_t int_bytes = up256((size_t)(2 + 2 * (int64_t)nbt * nbt) * sizeof(int32_t));
    void *ws = nullptr;
    int rc = ctx_workspace(ctx, kWsDag, task_bytes + int_bytes, &ws);
    if (rc) return rc;
    const uint64_t gen = ctx_workspace_gen(ctx, kWsDag);
    auto up = g_dag_uploaded.find(dev);
    if (up == g_dag_uploaded.end() || up->second.first != gen || up->second.second != e) {
        // the list stays alive in g_dag_lists while the copy is in flight
        if (!e->tasks.empty())
            FLAME_HIP(hipMemcpyAsync(ws, e->tasks.data(), e->tasks.size() * sizeof(int4), hipMemcpyHostToDevice, s));
        g_dag_uploaded[dev] = {gen, e};
    }
    int32_t *ints = reinterpret_cast<int32_t *>(static_cast<char *>(ws) + task_bytes);
    return launch_by_blocks(n, A, lda, static_cast<const int4 *>(ws), (int64_t)e->tasks.size(), nbt, ints, info, s);
}

void drop_dag_lists() {
    std::lock_guard<std::mutex> lk(g_dag_mu);
    g_dag_uploaded.clear();
}

}  // namespace flame

extern "C" {

int flame_factor_by_blocks(int32_t dtype, int64_t n, void *A, int64_t lda, const uint8_t *pattern, int32_t *info,
                           void *stream) {
    if (dtype != FLAME_F64) return dtype == FLAME_F32 ? FLAME_ERR_UNSUPPORTED : -1;
    if (n < 0 || n > ((int64_t)1 << 31) - 1) return -2;
    if (A == nullptr && n > 0) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (info == nullptr) return -6;
    return by_blocks_factor(n, static_cast<double *>(A), lda, pattern, info, static_cast<hipStream_t>(stream));
}

int flame_by_blocks_tasks(int64_t nbt, const uint8_t *pattern, int32_t *tasks, int64_t capacity, int64_t *count) {
    if (nbt < 0 || nbt > 4096) return -1;
    if (capacity < 0) return -4;
    if (count == nullptr) return -5;
    std::vector<uint8_t> pat;
    if (pattern != nullptr) {
        pat.assign((size_t)nbt * nbt, 0);
        for (int64_t i = 0; i < nbt; ++i)
            for (int64_t j = i; j < nbt; ++j) pat[(size_t)(i * nbt + j)] = (i == j || pattern[i * nbt + j]) ? 1 : 0;
    }
    const std::vector<int4> t = by_blocks_tasks((int)nbt, pat.empty() ? nullptr : pat.data());
    *count = (int64_t)t.size();
    if (tasks == nullptr) return FLAME_OK;
    if ((int64_t)t.size() > capacity) return -4;
    for (size_t q = 0; q < t.size(); ++q) {
        tasks[4 * q + 0] = t[q].x & 3;
        tasks[4 * q + 1] = t[q].x >> 2;
        tasks[4 * q + 2] = t[q].y;
        tasks[4 * q + 3] = t[q].z;
    }
    return FLAME_OK;
}

}  // extern "C"
