// flame_ichol_*: the paper's level(k) incomplete Cholesky factorization by
// blocks (Sec. "Symbolic factorization", Alg. symb_fact; Sec. "2D sparse
// partitioned-block matrix"; the numeric Cholesky-by-blocks of Fig.
// "sparse-chol").
//
// Symbolic phase, on the host (the paper reports its cost as small next to
// the numeric phase):
//   1. a nested dissection ordering (unless the caller gives one): the vertex
//      set is split by the middle level of a breadth-first level structure
//      rooted at a pseudo-peripheral vertex (that level separates the levels
//      before it from those after it); the two parts are ordered first, the
//      separator last; sets of at most `leaf` vertices (and sets that cannot
//      be split) are leaves, disconnected sets are ordered component by
//      component;
//   2. the level-k pattern of U by Hysom and Pothen's characterization: (i, j),
//      i < j, has level l when the shortest path from i to j whose inner
//      vertices are all numbered below i has l + 1 edges; a breadth-first
//      search from each i through lower-numbered vertices, k + 1 edges deep;
//   3. the 2D block layout: the ranges of the dissection (leaves and
//      separators, or the caller's ranges) cut into chunks of at most 128; a
//      block exists when the pattern has an entry in it.
// Numeric phase, on the device (k_dag.hip): the existing blocks live in a
// pool of 128 x 128 tiles; A's upper entries are scattered into it, and the
// task DAG of the block pattern runs with element masks (dropped fill).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <queue>
#include <vector>

#include "flame_internal.h"

namespace flame {
int launch_ichol_dag(double *pool, int64_t pool_elems, const double *vals, int64_t nnz_a, const int64_t *amap,
                     const int64_t *boff, const int32_t *bstart, const uint64_t *masks, const uint64_t *rowocc, int nbt,
                     const int4 *tasks, int64_t ntasks, int32_t *ints, int32_t *info, hipStream_t s);
int launch_gather_vals(int64_t nnz, const int64_t *map, const double *pool, double *out, hipStream_t s);
int launch_bsolve(bool forward, const double *pool, const int64_t *boff, const int32_t *bstart, int nbt,
                  const int32_t *lptr, const int32_t *lblk, double *y, int32_t *flags, int32_t *err, hipStream_t s);
int launch_spmv(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *x, const double *b,
                double *y, hipStream_t s);
int launch_permute(int64_t n, const int64_t *order, const double *src, double *dst, bool gather, hipStream_t s);
}  // namespace flame

using namespace flame;

namespace {

constexpr int kT = 128;          // tile order of the pool
constexpr int kMaxBlocks = 4096; // blocks per side (the futures are nbt^2 counters)

// ---- 1. nested dissection ----------------------------------------------------

struct Graph {
    int64_t n;
    std::vector<int64_t> xadj;
    std::vector<int32_t> adj;  // no self loops, symmetric
};

class Dissection {
  public:
    Dissection(const Graph &g, int leaf) : g_(g), leaf_(std::max(1, leaf)), mark_(g.n, -1), level_(g.n, -1) {}

    void run(std::vector<int64_t> &order, std::vector<int64_t> &ends) {
        std::vector<int32_t> all(g_.n);
        std::iota(all.begin(), all.end(), 0);
        rec(all);
        order.swap(order_);
        ends.swap(ends_);
    }

  private:
    void emit(std::vector<int32_t> v) {
        std::sort(v.begin(), v.end());
        for (int32_t x : v) order_.push_back(x);
        ends_.push_back((int64_t)order_.size());
    }

    // breadth-first levels of the vertices of set `id` reachable from `root`;
    // returns them in visiting order, level_[v] set
    std::vector<int32_t> bfs(int32_t root, int64_t id) {
        std::vector<int32_t> q{root};
        level_[root] = 0;
        stamp_++;
        seen(root);
        for (size_t h = 0; h < q.size(); ++h) {
            const int32_t v = q[h];
            for (int64_t e = g_.xadj[v]; e < g_.xadj[v + 1]; ++e) {
                const int32_t w = g_.adj[e];
                if (mark_[w] != id || is_seen(w)) continue;
                seen(w);
                level_[w] = level_[v] + 1;
                q.push_back(w);
            }
        }
        return q;
    }
    void seen(int32_t v) {
        if ((int64_t)visit_.size() < g_.n) visit_.assign(g_.n, 0);
        visit_[v] = stamp_;
    }
    bool is_seen(int32_t v) const { return visit_[v] == stamp_; }

    void rec(const std::vector<int32_t> &S) {
        if (S.empty()) return;
        const int64_t id = next_id_++;
        for (int32_t v : S) mark_[v] = id;
        if ((int64_t)S.size() <= leaf_) {
            emit(S);
            return;
        }
        // components
        std::vector<int32_t> comp = bfs(S[0], id);
        if (comp.size() < S.size()) {
            std::vector<int32_t> rest;
            for (int32_t v : S)
                if (!is_seen(v)) rest.push_back(v);
            rec(comp);
            rec(rest);
            return;
        }
        // pseudo-peripheral root: the last vertex reached, then again
        int32_t root = comp.back();
        for (int it = 0; it < 2; ++it) {
            for (int32_t v : S) mark_[v] = id;
            comp = bfs(root, id);
            root = comp.back();
        }
        const int32_t nlev = level_[comp.back()] + 1;
        std::vector<int64_t> count(nlev, 0);
        for (int32_t v : comp) count[level_[v]]++;
        int32_t m = 0;
        int64_t cum = 0;
        while (m < nlev && (cum += count[m]) * 2 < (int64_t)S.size()) ++m;
        if (m <= 0 || m >= nlev - 1) {  // no level to cut at
            emit(S);
            return;
        }
        std::vector<int32_t> a, b, sep;
        for (int32_t v : comp) (level_[v] < m ? a : level_[v] > m ? b : sep).push_back(v);
        rec(a);
        rec(b);
        emit(sep);
    }

    const Graph &g_;
    int64_t leaf_;
    std::vector<int64_t> mark_;
    std::vector<int32_t> level_;
    std::vector<int64_t> visit_;
    int64_t stamp_ = 0;
    int64_t next_id_ = 0;
    std::vector<int64_t> order_, ends_;
};

// ---- 2. level-k pattern ---------------------------------------------------------

// Rows of U (new numbering), columns increasing, the diagonal first.
void level_pattern(const Graph &g, int k, std::vector<int64_t> &urp, std::vector<int32_t> &uci) {
    const int64_t n = g.n;
    std::vector<int64_t> stamp(n, -1);
    std::vector<int32_t> frontier, next, row;
    urp.assign(n + 1, 0);
    uci.clear();
    for (int64_t i = 0; i < n; ++i) {
        row.clear();
        row.push_back((int32_t)i);
        stamp[i] = i;
        frontier.assign(1, (int32_t)i);
        // depth d: the vertices of the frontier end paths with d inner vertices
        for (int d = 0; d <= k && !frontier.empty(); ++d) {
            next.clear();
            for (int32_t v : frontier)
                for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
                    const int32_t w = g.adj[e];
                    if (stamp[w] == i) continue;
                    stamp[w] = i;
                    if (w > i)
                        row.push_back(w);  // level d
                    else if (d + 1 <= k)
                        next.push_back(w);  // an inner vertex, d + 1 of them so far
                }
            frontier.swap(next);
        }
        std::sort(row.begin() + 1, row.end());
        uci.insert(uci.end(), row.begin(), row.end());
        urp[i + 1] = (int64_t)uci.size();
    }
}

// ---- 3. task list of a sparse block pattern ----------------------------------------

// The order of by_blocks_tasks (k_dag.hip) over the existing blocks only:
// rows[k] = the existing blocks j > k of block row k, increasing.
std::vector<int4> sparse_tasks(int nbt, const std::vector<std::vector<int32_t>> &rows,
                               const std::vector<int32_t> &bid) {
    auto ex = [&](int i, int j) { return i == j || bid[(int64_t)i * nbt + j] >= 0; };
    std::vector<int4> out;
    std::vector<std::vector<int64_t>> upd_of_k(nbt);  // positions of the updates of iteration k
    auto upd_row = [&](int k, int i) {
        if (k < 0 || i >= nbt || !ex(k, i)) return;
        const auto &R = rows[k];
        for (auto it = std::lower_bound(R.begin(), R.end(), i); it != R.end(); ++it) {
            const int j = *it;
            if (!ex(i, j)) continue;
            upd_of_k[k].push_back((int64_t)out.size());
            out.push_back(int4{2 | (k << 2), i, j, 0});
        }
    };
    std::vector<int64_t> chol_pos(nbt), trsm_first(nbt);
    for (int r = 0; r < nbt; ++r) {
        chol_pos[r] = (int64_t)out.size();
        out.push_back(int4{0 | (r << 2), r, r, 0});
        trsm_first[r] = (int64_t)out.size();
        for (int j : rows[r]) out.push_back(int4{1 | (r << 2), r, j, 0});
        upd_row(r - 1, r + 1);
        upd_row(r, r + 1);
        if (r >= 1)
            for (auto it = std::lower_bound(rows[r - 1].begin(), rows[r - 1].end(), r + 2); it != rows[r - 1].end(); ++it)
                upd_row(r - 1, *it);
    }
    // need: the updates of a block from earlier iterations
    std::vector<int32_t> cnt(bid.size(), 0);
    for (int k = 0; k < nbt; ++k)
        for (int64_t q : upd_of_k[k]) {
            int4 &t = out[q];
            t.w = cnt[(int64_t)t.y * nbt + t.z]++;
        }
    for (int r = 0; r < nbt; ++r) {
        out[chol_pos[r]].w = cnt[(int64_t)r * nbt + r];
        for (size_t q = 0; q < rows[r].size(); ++q) out[trsm_first[r] + q].w = cnt[(int64_t)r * nbt + rows[r][q]];
    }
    return out;
}

// The claim order for a sparse pattern.  Any order in which every task
// follows the tasks it waits for keeps the launch progressing; for a nested
// dissection the by-iteration order above leaves workgroups waiting on
// separator tasks claimed long before their subtrees are done.  So the list is
// reordered by a simulated list schedule: tasks with estimated costs (`cost`,
// per type) on `workers` workgroups, a ready task with the longest remaining
// path to the end first, listed by simulated start time.  The per-block update
// chains keep their iteration order (each update waits for the previous one).
std::vector<int4> schedule_order(const std::vector<int4> &tasks, int nbt, const std::vector<int32_t> &bid,
                                 int64_t nblocks, int workers, const double cost[3]) {
    const int64_t T = (int64_t)tasks.size();
    std::vector<int64_t> chol_of(nbt, -1);
    std::vector<std::vector<int64_t>> deps(T);
    // per existing block: its TRSM and the updates into it, by need
    auto id = [&](int i, int j) { return bid[(size_t)i * nbt + j]; };
    std::vector<std::vector<std::pair<int32_t, int64_t>>> upd_into(nblocks);
    std::vector<int64_t> trsm_of(nblocks, -1);
    for (int64_t t = 0; t < T; ++t) {
        const int type = tasks[t].x & 3, k = tasks[t].x >> 2;
        if (type == 0) chol_of[k] = t;
        else if (type == 1) trsm_of[id(k, tasks[t].z)] = t;
        else upd_into[id(tasks[t].y, tasks[t].z)].push_back({tasks[t].w, t});
    }
    for (auto &v : upd_into) std::sort(v.begin(), v.end());
    auto last_upd = [&](int i, int j) -> int64_t {
        const auto &v = upd_into[id(i, j)];
        return v.empty() ? -1 : v.back().second;
    };
    for (int64_t t = 0; t < T; ++t) {
        const int type = tasks[t].x & 3, k = tasks[t].x >> 2, i = tasks[t].y, j = tasks[t].z;
        auto add = [&](int64_t d) {
            if (d >= 0) deps[t].push_back(d);
        };
        if (type == 0) {
            add(last_upd(k, k));
        } else if (type == 1) {
            add(chol_of[k]);
            add(last_upd(k, j));
        } else {
            add(trsm_of[id(k, i)]);
            add(trsm_of[id(k, j)]);
            const int need = tasks[t].w;
            if (need > 0) add(upd_into[id(i, j)][need - 1].second);
        }
    }
    std::vector<std::vector<int64_t>> succ(T);
    std::vector<int32_t> indeg(T, 0);
    for (int64_t t = 0; t < T; ++t)
        for (int64_t d : deps[t]) {
            succ[d].push_back(t);
            ++indeg[t];
        }
    // longest path to the end (the list is already a topological order)
    std::vector<double> bl(T, 0.0);
    for (int64_t t = T - 1; t >= 0; --t) {
        double m = 0.0;
        for (int64_t q : succ[t]) m = std::max(m, bl[q]);
        bl[t] = cost[tasks[t].x & 3] + m;
    }
    // list scheduling
    typedef std::pair<double, int64_t> Item;
    std::priority_queue<Item> ready;  // highest remaining path first
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> running;  // by finish time
    for (int64_t t = 0; t < T; ++t)
        if (indeg[t] == 0) ready.push({bl[t], -t});
    std::vector<int4> out;
    out.reserve(T);
    double now = 0.0;
    int busy = 0;
    while ((int64_t)out.size() < T) {
        while (busy < workers && !ready.empty()) {
            const int64_t t = -ready.top().second;
            ready.pop();
            out.push_back(tasks[t]);
            running.push({now + cost[tasks[t].x & 3], t});
            ++busy;
        }
        if (running.empty()) break;  // (cannot happen for a valid list)
        const Item f = running.top();
        running.pop();
        --busy;
        now = f.first;
        for (int64_t q : succ[f.second])
            if (--indeg[q] == 0) ready.push({bl[q], -q});
    }
    return out;
}

}  // namespace

struct flame_ichol_plan_s {
    int dev = -1;  // the device holding the plan's buffers (bound by the first factor call)
    int64_t n = 0, nnz_a = 0, nnz_u = 0;
    int32_t level = 0;
    int nbt = 0;
    int64_t nblocks = 0;
    std::vector<int64_t> order, bounds;
    std::vector<int64_t> urp;
    std::vector<int32_t> uci;
    std::vector<uint8_t> pattern;  // nbt x nbt, upper
    std::vector<int4> tasks;
    // host copies of what goes to the device
    std::vector<uint64_t> h_masks, h_rowocc;
    // the input pattern (for the sparse product of PCG) and the block lists of
    // the triangular solves
    std::vector<int64_t> h_rp;
    std::vector<int32_t> h_ci;
    bool full_sym = false;  // both triangles stored (needed by the product)
    std::vector<int32_t> h_fptr, h_fblk, h_bptr, h_bblk;
    std::vector<int64_t> h_boff, h_amap, h_umap;
    std::vector<int32_t> h_bstart;
    double *pool = nullptr;
    uint64_t *masks = nullptr;
    uint64_t *rowocc = nullptr;
    int64_t *boff = nullptr;
    int32_t *bstart = nullptr;
    int4 *dtasks = nullptr;
    int32_t *ints = nullptr;
    int64_t *amap = nullptr;
    int64_t *umap = nullptr;
    // solves and PCG (allocated with the rest)
    int64_t *d_order = nullptr, *d_rp = nullptr;
    int32_t *d_ci = nullptr, *d_fptr = nullptr, *d_fblk = nullptr, *d_bptr = nullptr, *d_bblk = nullptr;
    int32_t *d_flags = nullptr, *d_err = nullptr;
    double *d_vec = nullptr;  // r, z, p, q, t (n each) and scalars rho, rho_old, pq, rr
};

namespace {

void free_plan(flame_ichol_plan_s *p) {
    if (p == nullptr) return;
    if (p->dev < 0) {
        delete p;
        return;
    }
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != p->dev) (void)hipSetDevice(p->dev);
    for (void *q : {(void *)p->pool, (void *)p->masks, (void *)p->rowocc, (void *)p->boff, (void *)p->bstart,
                    (void *)p->dtasks, (void *)p->ints, (void *)p->amap, (void *)p->umap, (void *)p->d_order,
                    (void *)p->d_rp, (void *)p->d_ci, (void *)p->d_fptr, (void *)p->d_fblk, (void *)p->d_bptr,
                    (void *)p->d_bblk, (void *)p->d_flags, (void *)p->d_err, (void *)p->d_vec})
        if (q != nullptr) (void)hipFree(q);
    if (cur != p->dev) (void)hipSetDevice(cur);
    delete p;
}

template <typename T>
int upload(T **dst, const std::vector<T> &src) {
    const size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
    if (hipMalloc((void **)dst, bytes) != hipSuccess) return FLAME_ERR_NOMEM;
    if (!src.empty() && hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return FLAME_ERR_HIP;
    return FLAME_OK;
}

// Uploads the plan to the current device on first use (the symbolic phase
// needs no device); later calls must be on that device.
int ensure_device(flame_ichol_plan_s *p) {
    int cur = 0;
    FLAME_HIP(hipGetDevice(&cur));
    if (p->dev >= 0) return cur == p->dev ? FLAME_OK : FLAME_ERR_UNSUPPORTED;
    p->dev = cur;
    int rc = FLAME_OK;
    const size_t pool_bytes = std::max<int64_t>(1, p->nblocks) * (size_t)kT * kT * sizeof(double);
    if (hipMalloc((void **)&p->pool, pool_bytes) != hipSuccess) rc = FLAME_ERR_NOMEM;
    if (!rc) rc = upload(&p->masks, p->h_masks);
    if (!rc) rc = upload(&p->rowocc, p->h_rowocc);
    if (!rc) rc = upload(&p->boff, p->h_boff);
    if (!rc) rc = upload(&p->bstart, p->h_bstart);
    if (!rc) rc = upload(&p->dtasks, p->tasks);
    if (!rc) rc = upload(&p->amap, p->h_amap);
    if (!rc) rc = upload(&p->umap, p->h_umap);
    if (!rc && hipMalloc((void **)&p->ints, (3 + 2 * (size_t)p->nbt * p->nbt) * sizeof(int32_t)) != hipSuccess)
        rc = FLAME_ERR_NOMEM;
    if (!rc) rc = upload(&p->d_order, p->order);
    if (!rc) rc = upload(&p->d_rp, p->h_rp);
    if (!rc) rc = upload(&p->d_ci, p->h_ci);
    if (!rc) rc = upload(&p->d_fptr, p->h_fptr);
    if (!rc) rc = upload(&p->d_fblk, p->h_fblk);
    if (!rc) rc = upload(&p->d_bptr, p->h_bptr);
    if (!rc) rc = upload(&p->d_bblk, p->h_bblk);
    if (!rc && hipMalloc((void **)&p->d_flags, std::max(1, p->nbt) * sizeof(int32_t)) != hipSuccess) rc = FLAME_ERR_NOMEM;
    if (!rc && hipMalloc((void **)&p->d_err, sizeof(int32_t)) != hipSuccess) rc = FLAME_ERR_NOMEM;
    if (!rc && hipMalloc((void **)&p->d_vec, (5 * (size_t)std::max<int64_t>(1, p->n) + 8) * sizeof(double)) != hipSuccess)
        rc = FLAME_ERR_NOMEM;
    if (rc) {  // back to unbound: a later call tries again
        for (void **q : {(void **)&p->pool, (void **)&p->masks, (void **)&p->rowocc, (void **)&p->boff,
                         (void **)&p->bstart, (void **)&p->dtasks, (void **)&p->ints, (void **)&p->amap,
                         (void **)&p->umap, (void **)&p->d_order, (void **)&p->d_rp, (void **)&p->d_ci,
                         (void **)&p->d_fptr, (void **)&p->d_fblk, (void **)&p->d_bptr, (void **)&p->d_bblk,
                         (void **)&p->d_flags, (void **)&p->d_err, (void **)&p->d_vec})
            if (*q != nullptr) {
                (void)hipFree(*q);
                *q = nullptr;
            }
        p->dev = -1;
    }
    return rc;
}

}  // namespace

extern "C" {

int flame_ichol_analyze(int64_t n, const int64_t *rp, const int32_t *ci, int32_t level, const int64_t *order,
                        const int64_t *bounds, int64_t nranges, int32_t leaf, flame_ichol_plan *plan_out) {
    if (n < 0 || n > ((int64_t)1 << 31) - 1) return -1;
    if (rp == nullptr) return -2;
    if (ci == nullptr && n > 0 && rp[n] > 0) return -3;
    if (level < 0) return -4;
    if (bounds != nullptr && order == nullptr) return -6;
    if (bounds != nullptr && nranges < 1) return -7;
    if (leaf < 0) return -8;
    if (plan_out == nullptr) return -9;
    *plan_out = nullptr;
    if (rp[0] != 0) return -2;
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return -2;
    for (int64_t e = 0; e < rp[n]; ++e)
        if (ci[e] < 0 || ci[e] >= n) return -3;
    // the graph of A: symmetric, no self loops
    Graph g;
    g.n = n;
    {
        std::vector<std::vector<int32_t>> nb(n);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
                const int32_t j = ci[e];
                if (j == i) continue;
                nb[i].push_back(j);
                nb[j].push_back((int32_t)i);
            }
        g.xadj.assign(n + 1, 0);
        for (int64_t i = 0; i < n; ++i) {
            auto &v = nb[i];
            std::sort(v.begin(), v.end());
            v.erase(std::unique(v.begin(), v.end()), v.end());
            g.xadj[i + 1] = g.xadj[i] + (int64_t)v.size();
        }
        g.adj.reserve(g.xadj[n]);
        for (auto &v : nb) g.adj.insert(g.adj.end(), v.begin(), v.end());
    }
    auto *p = new flame_ichol_plan_s();
    p->n = n;
    p->nnz_a = rp[n];
    p->level = level;
    p->h_rp.assign(rp, rp + n + 1);
    p->h_ci.assign(ci, ci + rp[n]);
    {
        int64_t offdiag = 0;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) offdiag += (ci[e] != i);
        p->full_sym = (offdiag == (int64_t)g.adj.size());  // every edge stored in both directions
    }
    // 1. ordering and ranges
    std::vector<int64_t> ends;
    if (order != nullptr) {
        p->order.assign(order, order + n);
        std::vector<uint8_t> hit(n, 0);
        for (int64_t v : p->order) {
            if (v < 0 || v >= n || hit[v]) {
                delete p;
                return -5;
            }
            hit[v] = 1;
        }
        if (bounds != nullptr) {
            if (bounds[0] != 0 || bounds[nranges] != n) {
                delete p;
                return -6;
            }
            for (int64_t r = 0; r < nranges; ++r) {
                if (bounds[r + 1] <= bounds[r]) {
                    delete p;
                    return -6;
                }
                ends.push_back(bounds[r + 1]);
            }
        } else {
            for (int64_t e = kT; e < n; e += kT) ends.push_back(e);
            if (n > 0) ends.push_back(n);
        }
    } else {
        Dissection(g, leaf > 0 ? leaf : kT).run(p->order, ends);
    }
    // ranges cut into chunks of at most 128
    p->bounds.assign(1, 0);
    int64_t start = 0;
    for (int64_t e : ends) {
        const int64_t len = e - start;
        const int64_t pieces = (len + kT - 1) / kT;
        for (int64_t q = 1; q <= pieces; ++q) p->bounds.push_back(start + (len * q) / pieces);
        start = e;
    }
    p->nbt = (int)(p->bounds.size() - 1);
    if (p->nbt > kMaxBlocks) {
        delete p;
        return FLAME_ERR_UNSUPPORTED;
    }
    // the graph in the new numbering
    std::vector<int64_t> inv(n);
    for (int64_t v = 0; v < n; ++v) inv[p->order[v]] = v;
    Graph h;
    h.n = n;
    h.xadj.assign(n + 1, 0);
    h.adj.resize(g.adj.size());
    for (int64_t v = 0; v < n; ++v) {
        const int64_t old = p->order[v];
        h.xadj[v + 1] = h.xadj[v] + (g.xadj[old + 1] - g.xadj[old]);
    }
    for (int64_t v = 0; v < n; ++v) {
        const int64_t old = p->order[v];
        int64_t o = h.xadj[v];
        for (int64_t e = g.xadj[old]; e < g.xadj[old + 1]; ++e) h.adj[o++] = (int32_t)inv[g.adj[e]];
    }
    // 2. the level-k pattern
    level_pattern(h, level, p->urp, p->uci);
    p->nnz_u = (int64_t)p->uci.size();
    // 3. blocks
    const int nbt = p->nbt;
    std::vector<int32_t> blk(n);
    for (int b = 0; b < nbt; ++b)
        for (int64_t i = p->bounds[b]; i < p->bounds[b + 1]; ++i) blk[i] = b;
    p->pattern.assign((size_t)nbt * nbt, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = p->urp[i]; e < p->urp[i + 1]; ++e) p->pattern[(size_t)blk[i] * nbt + blk[p->uci[e]]] = 1;
    for (int b = 0; b < nbt; ++b) p->pattern[(size_t)b * nbt + b] = 1;
    std::vector<int32_t> bid((size_t)nbt * nbt, -1);
    std::vector<std::vector<int32_t>> rows(nbt);
    int64_t nblocks = 0;
    for (int bi = 0; bi < nbt; ++bi)
        for (int bj = bi; bj < nbt; ++bj)
            if (p->pattern[(size_t)bi * nbt + bj]) {
                bid[(size_t)bi * nbt + bj] = (int32_t)nblocks++;
                if (bj > bi) rows[bi].push_back(bj);
            }
    p->nblocks = nblocks;
    // block lists of the solves: forward, for block column i the q < i with
    // (q, i); backward, for block row i the j > i with (i, j)
    {
        std::vector<std::vector<int32_t>> cols(nbt);
        for (int bi = 0; bi < nbt; ++bi)
            for (int bj : rows[bi]) cols[bj].push_back(bi);
        p->h_fptr.assign(1, 0);
        p->h_bptr.assign(1, 0);
        for (int b = 0; b < nbt; ++b) {
            p->h_fblk.insert(p->h_fblk.end(), cols[b].begin(), cols[b].end());
            p->h_fptr.push_back((int32_t)p->h_fblk.size());
            p->h_bblk.insert(p->h_bblk.end(), rows[b].begin(), rows[b].end());
            p->h_bptr.push_back((int32_t)p->h_bblk.size());
        }
    }
    {
        // estimated microseconds per task on one workgroup: CHOL, TRSM, update
        const double cost[3] = {100.0, 60.0, 30.0};
        p->tasks = schedule_order(sparse_tasks(nbt, rows, bid), nbt, bid, nblocks, 256, cost);
    }
    // tile offsets, masks, maps
    std::vector<int64_t> boff((size_t)nbt * nbt, -1);
    for (size_t q = 0; q < bid.size(); ++q)
        if (bid[q] >= 0) boff[q] = (int64_t)bid[q] * kT * kT;
    std::vector<uint64_t> masks((size_t)nblocks * 2 * kT, 0);
    std::vector<int64_t> umap(p->nnz_u);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = p->urp[i]; e < p->urp[i + 1]; ++e) {
            const int64_t j = p->uci[e];
            const int bi = blk[i], bj = blk[j];
            const int64_t r = i - p->bounds[bi], c = j - p->bounds[bj];
            const int64_t t = bid[(size_t)bi * nbt + bj];
            masks[(size_t)t * 2 * kT + 2 * c + (r >> 6)] |= (uint64_t)1 << (r & 63);
            umap[e] = boff[(size_t)bi * nbt + bj] + r + c * kT;
        }
    std::vector<int64_t> amap(p->nnz_a, -1);
    for (int64_t io = 0; io < n; ++io)
        for (int64_t e = rp[io]; e < rp[io + 1]; ++e) {
            const int64_t i = inv[io], j = inv[ci[e]];
            if (i > j) continue;
            const int bi = blk[i], bj = blk[j];
            amap[e] = boff[(size_t)bi * nbt + bj] + (i - p->bounds[bi]) + (j - p->bounds[bj]) * kT;
        }
    // row occupancy per tile: the OR of its columns' mask words
    p->h_rowocc.assign((size_t)nblocks * 2, 0);
    for (int64_t t = 0; t < nblocks; ++t)
        for (int c = 0; c < kT; ++c) {
            p->h_rowocc[2 * t] |= masks[(size_t)t * 2 * kT + 2 * c];
            p->h_rowocc[2 * t + 1] |= masks[(size_t)t * 2 * kT + 2 * c + 1];
        }
    p->h_masks.swap(masks);
    p->h_boff.swap(boff);
    p->h_amap.swap(amap);
    p->h_umap.swap(umap);
    p->h_bstart.assign(p->bounds.begin(), p->bounds.end());
    *plan_out = p;
    return FLAME_OK;
}

int flame_ichol_stats(flame_ichol_plan plan, flame_ichol_stats_t *st) {
    if (plan == nullptr) return -1;
    if (st == nullptr) return -2;
    st->n = plan->n;
    st->nnz_a = plan->nnz_a;
    st->nnz_u = plan->nnz_u;
    st->nbt = plan->nbt;
    st->nblocks = plan->nblocks;
    st->ntasks = (int64_t)plan->tasks.size();
    st->pool_bytes = plan->nblocks * (int64_t)kT * kT * (int64_t)sizeof(double);
    double f = 0.0;  // multiply-adds of the incomplete factorization: per pivot k, one per (i <= j) pair of
                     // row k whose target (i, j) is in the pattern, plus the row's scaling
    {
        const int64_t n = plan->n;
        std::vector<int64_t> pos(n, -1);
        int64_t stamp = 0;
        for (int64_t k = 0; k < n; ++k) {
            const int64_t b = plan->urp[k], e = plan->urp[k + 1];
            f += (double)(e - b);  // sqrt and the scaling of the row
            for (int64_t qi = b + 1; qi < e; ++qi) {
                const int64_t i = plan->uci[qi];
                ++stamp;  // marks row i's columns for this (k, i) only
                for (int64_t q = plan->urp[i]; q < plan->urp[i + 1]; ++q) pos[plan->uci[q]] = stamp;
                for (int64_t qj = qi; qj < e; ++qj)
                    if (pos[plan->uci[qj]] == stamp) f += 2.0;
            }
        }
    }
    st->flops = f;
    return FLAME_OK;
}

int flame_ichol_structure(flame_ichol_plan plan, int64_t *order, int64_t *bounds, int64_t *urp, int32_t *uci,
                          uint8_t *pattern, int32_t *tasks) {
    if (plan == nullptr) return -1;
    if (order) std::memcpy(order, plan->order.data(), plan->order.size() * sizeof(int64_t));
    if (bounds) std::memcpy(bounds, plan->bounds.data(), plan->bounds.size() * sizeof(int64_t));
    if (urp) std::memcpy(urp, plan->urp.data(), plan->urp.size() * sizeof(int64_t));
    if (uci) std::memcpy(uci, plan->uci.data(), plan->uci.size() * sizeof(int32_t));
    if (pattern) std::memcpy(pattern, plan->pattern.data(), plan->pattern.size());
    if (tasks)
        for (size_t q = 0; q < plan->tasks.size(); ++q) {
            tasks[4 * q + 0] = plan->tasks[q].x & 3;
            tasks[4 * q + 1] = plan->tasks[q].x >> 2;
            tasks[4 * q + 2] = plan->tasks[q].y;
            tasks[4 * q + 3] = plan->tasks[q].z;
        }
    return FLAME_OK;
}

int flame_ichol_factor(flame_ichol_plan plan, const double *vals, int32_t *info, void *stream) {
    if (plan == nullptr) return -1;
    if (vals == nullptr && plan->nnz_a > 0) return -2;
    if (info == nullptr) return -3;
    const int rc = ensure_device(plan);
    if (rc) return rc;
    return launch_ichol_dag(plan->pool, plan->nblocks * (int64_t)kT * kT, vals, plan->nnz_a, plan->amap, plan->boff,
                            plan->bstart, plan->masks, plan->rowocc, plan->nbt, plan->dtasks, (int64_t)plan->tasks.size(),
                            plan->ints, info, static_cast<hipStream_t>(stream));
}

int flame_ichol_values(flame_ichol_plan plan, double *uvals, void *stream) {
    if (plan == nullptr) return -1;
    if (uvals == nullptr && plan->nnz_u > 0) return -2;
    const int rc = ensure_device(plan);
    if (rc) return rc;
    return launch_gather_vals(plan->nnz_u, plan->umap, plan->pool, uvals, static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace {

// z := P^T (U^T U)^{-1} P r (device vectors, original numbering) through t.
int apply_precond(flame_ichol_plan_s *p, const double *r, double *z, double *t, hipStream_t s) {
    int rc = launch_permute(p->n, p->d_order, r, t, true, s);
    if (!rc) rc = launch_bsolve(true, p->pool, p->boff, p->bstart, p->nbt, p->d_fptr, p->d_fblk, t, p->d_flags,
                                p->d_err, s);
    if (!rc) rc = launch_bsolve(false, p->pool, p->boff, p->bstart, p->nbt, p->d_bptr, p->d_bblk, t, p->d_flags,
                                p->d_err, s);
    if (!rc) rc = launch_permute(p->n, p->d_order, t, z, false, s);
    return rc;
}

}  // namespace

extern "C" {

int flame_ichol_apply(flame_ichol_plan plan, const double *r, double *z, void *stream) {
    if (plan == nullptr) return -1;
    if (r == nullptr && plan->n > 0) return -2;
    if (z == nullptr && plan->n > 0) return -3;
    int rc = ensure_device(plan);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = launch_zero_i32(plan->d_err, 1, s);
    if (rc) return rc;
    return apply_precond(plan, r, z, plan->d_vec + 4 * plan->n, s);
}

int flame_ichol_pcg(flame_ichol_plan plan, const double *vals, const double *b, double *x, const flame_pcg_opts_t *opts,
                    flame_pcg_report_t *report, void *stream) {
    if (plan == nullptr) return -1;
    const int64_t n = plan->n;
    if (vals == nullptr && plan->nnz_a > 0) return -2;
    if (b == nullptr && n > 0) return -3;
    if (x == nullptr && n > 0) return -4;
    const double tol = opts ? opts->tol : 1e-10;
    const int32_t max_iter = opts ? opts->max_iter : 1000;
    if (!(tol > 0.0) || max_iter < 0) return -5;
    if (opts && (opts->reserved[0] || opts->reserved[1])) return -5;
    if (!plan->full_sym) return FLAME_ERR_UNSUPPORTED;
    int rc = ensure_device(plan);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    flame_pcg_report_t rep{0, FLAME_OK, 0.0, 0.0};
    if (n == 0) {
        if (report) *report = rep;
        return FLAME_OK;
    }
    double *r = plan->d_vec, *z = r + n, *pv = z + n, *q = pv + n, *t = q + n;
    double *sc = t + n;  // rho, rho_old, pq, rr, bb
    double *rho = sc, *rho_old = sc + 1, *pq = sc + 2, *rr = sc + 3, *bb = sc + 4;
    rc = launch_zero_i32(plan->d_err, 1, s);
    if (!rc) rc = launch_dot_cols(n, 1, b, n, b, n, bb, s);
    if (!rc) rc = launch_spmv(n, plan->d_rp, plan->d_ci, vals, x, b, r, s);  // r = b - A x
    if (!rc) rc = launch_dot_cols(n, 1, r, n, r, n, rr, s);
    double host[2] = {0.0, 0.0};
    if (!rc) FLAME_HIP(hipMemcpyAsync(host, rr, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    if (!rc) FLAME_HIP(hipStreamSynchronize(s));
    if (rc) return rc;
    const double nb = std::sqrt(host[1]);
    rep.bnorm = nb;
    rep.relres = nb > 0.0 ? std::sqrt(host[0]) / nb : 0.0;
    if (nb == 0.0 || rep.relres <= tol) {
        if (report) *report = rep;
        return FLAME_OK;
    }
    bool first = true;
    int32_t it = 0;
    while (it < max_iter) {
        rc = apply_precond(plan, r, z, t, s);
        if (!rc && !first) FLAME_HIP(hipMemcpyAsync(rho_old, rho, sizeof(double), hipMemcpyDeviceToDevice, s));
        if (!rc) rc = launch_dot_cols(n, 1, r, n, z, n, rho, s);
        if (!rc) rc = launch_cg_direction(n, 1, z, n, pv, n, rho, rho_old, first, s);
        if (!rc) rc = launch_spmv(n, plan->d_rp, plan->d_ci, vals, pv, nullptr, q, s);
        if (!rc) rc = launch_dot_cols(n, 1, pv, n, q, n, pq, s);
        if (!rc) rc = launch_cg_step(n, 1, x, n, r, n, pv, n, q, n, rho, pq, s);
        if (!rc) rc = launch_dot_cols(n, 1, r, n, r, n, rr, s);
        int32_t err = 0;
        if (!rc) FLAME_HIP(hipMemcpyAsync(host, rr, sizeof(double), hipMemcpyDeviceToHost, s));
        if (!rc) FLAME_HIP(hipMemcpyAsync(&err, plan->d_err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        if (!rc) FLAME_HIP(hipStreamSynchronize(s));
        if (rc) return rc;
        if (err != 0) return FLAME_ERR_HIP;  // a solve gave up waiting
        first = false;
        ++it;
        rep.relres = std::sqrt(host[0]) / nb;
        if (!(rep.relres > tol)) break;  // converged (or NaN: reported below)
    }
    rep.iters = it;
    rep.status = (rep.relres <= tol) ? FLAME_OK : FLAME_ERR_NOT_CONVERGED;
    if (report) *report = rep;
    return FLAME_OK;
}

int flame_ichol_destroy(flame_ichol_plan plan) {
    if (plan == nullptr) return -1;
    free_plan(plan);
    return FLAME_OK;
}

}  // extern "C"
