// Host analysis: maximin ordering, sparsity pattern S and the level schedule.
//
// Ordering and pattern follow Section 2.3 (maximin ordering; S_rho with the
// max-rule, or the min-rule of Section 6.2).  Like the paper's SortSparse
// algorithm (Section 4.1) the ordering is produced with a mutable max-heap of
// current distances, but the candidate points to update are found with a k-d
// tree search around the newly selected point instead of parent/child lists:
// a subtree is entered only if its box may hold an unselected point closer than
// that point's current distance (per-node upper bounds of those distances).
// With enough points and threads, the ordering takes batches of heap
// candidates at once and applies their updates on several threads; the output
// is the same (see maximin_parallel).  Every comparison that decides the output uses the same
// floating-point expression as the definition, so the result is exactly the
// greedy maximin ordering and exactly S_rho:
//   dist(a,b) = sqrt(sum_t (a_t - b_t)^2), summed over t ascending, no fma;
//   (a,b) in S  <=>  dist <= rho * l.
// Tree pruning uses a box lower bound evaluated with the same operation
// sequence; rounding is monotone, so the bound never exceeds the distance of
// any point in the box and no candidate is lost.
//
// Compiled with -ffp-contract=off.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <climits>
#include <condition_variable>
#include <mutex>
#include <limits>
#include <thread>
#include <vector>

#include "plan.h"

namespace kc {
namespace {


int resolve_threads(int nthreads) {
    if (nthreads > 0) return nthreads;
    unsigned h = std::thread::hardware_concurrency();
    return h ? int(h) : 1;
}

// Dynamic parallel loop over [0, count) in chunks.
template <class F>
void parallel_for(int nthreads, int64_t count, int64_t chunk, F&& fn) {
    if (count <= 0) return;
    nthreads = std::max(1, std::min<int>(nthreads, int((count + chunk - 1) / chunk)));
    if (nthreads == 1) {
        fn(int64_t(0), count, 0);
        return;
    }
    std::atomic<int64_t> next{0};
    auto work = [&](int tid) {
        for (;;) {
            int64_t b = next.fetch_add(chunk);
            if (b >= count) break;
            fn(b, std::min(count, b + chunk), tid);
        }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nthreads; ++t) pool.emplace_back(work, t);
    work(0);
    for (auto& th : pool) th.join();
}

inline double dist(const double* a, const double* b, int d) {
    double s = 0.0;
    for (int t = 0; t < d; ++t) {
        double df = a[t] - b[t];
        s += df * df;
    }
    return std::sqrt(s);
}

// k-d tree over n points (ids 0..n-1 index the point array).
struct KDTree {
    struct Node {
        int32_t begin, end;   // range in idx
        int32_t left, right;  // children, -1 for a leaf
        int32_t minid, maxid; // smallest / largest point id in the subtree
    };
    int d = 0;
    const double* pts = nullptr;
    std::vector<int32_t> idx;
    std::vector<Node> nodes;
    std::vector<double> lo, hi;  // per node, d each

    static constexpr int kLeaf = 16;

    // Nodes of a subtree in pre-order (ids local to it) with their boxes.
    struct Sub {
        std::vector<Node> nodes;
        std::vector<double> lo, hi;
    };

    // From kParallelBuild points on, the two halves of the top levels are built
    // on separate threads (each works on its own range of idx) and appended in
    // pre-order, so the tree is the one the one-thread build gives.
    static constexpr int64_t kParallelBuild = 65536;

    void build(const double* p, int64_t n, int dim, int nthreads = 1) {
        pts = p;
        d = dim;
        idx.resize(n);
        for (int64_t i = 0; i < n; ++i) idx[i] = int32_t(i);
        int par_depth = 0;
        if (n >= kParallelBuild)
            while ((1 << par_depth) < nthreads && par_depth < 4) ++par_depth;
        Sub root;
        root.nodes.reserve(size_t(2 * (n / kLeaf + 1)));
        build_node(0, int32_t(n), 0, par_depth, root);
        nodes = std::move(root.nodes);
        lo = std::move(root.lo);
        hi = std::move(root.hi);
    }

    int32_t build_node(int32_t b, int32_t e, int depth, int par_depth, Sub& s) {
        int32_t id = int32_t(s.nodes.size());
        s.nodes.push_back(Node{b, e, -1, -1, 0, 0});
        s.lo.resize(size_t(s.nodes.size()) * d);
        s.hi.resize(size_t(s.nodes.size()) * d);
        double* L = &s.lo[size_t(id) * d];
        double* H = &s.hi[size_t(id) * d];
        for (int t = 0; t < d; ++t) {
            L[t] = std::numeric_limits<double>::infinity();
            H[t] = -std::numeric_limits<double>::infinity();
        }
        int32_t mn = idx[b], mx = idx[b];
        for (int32_t i = b; i < e; ++i) {
            const double* q = pts + size_t(idx[i]) * d;
            for (int t = 0; t < d; ++t) {
                L[t] = std::min(L[t], q[t]);
                H[t] = std::max(H[t], q[t]);
            }
            mn = std::min(mn, idx[i]);
            mx = std::max(mx, idx[i]);
        }
        s.nodes[id].minid = mn;
        s.nodes[id].maxid = mx;
        if (e - b <= kLeaf) return id;
        int ax = 0;
        double w = -1.0;
        for (int t = 0; t < d; ++t)
            if (H[t] - L[t] > w) {
                w = H[t] - L[t];
                ax = t;
            }
        if (!(w > 0.0)) return id;  // all points coincide: keep as one leaf
        int32_t mid = b + (e - b) / 2;
        std::nth_element(idx.begin() + b, idx.begin() + mid, idx.begin() + e, [&](int32_t u, int32_t v) {
            double a = pts[size_t(u) * d + ax], c = pts[size_t(v) * d + ax];
            return a < c || (a == c && u < v);
        });
        if (depth < par_depth) {
            Sub right;
            std::thread th([&] { build_node(mid, e, depth + 1, par_depth, right); });
            const int32_t l = build_node(b, mid, depth + 1, par_depth, s);
            th.join();
            const int32_t off = int32_t(s.nodes.size());
            for (Node nd : right.nodes) {
                if (nd.left >= 0) {
                    nd.left += off;
                    nd.right += off;
                }
                s.nodes.push_back(nd);
            }
            s.lo.insert(s.lo.end(), right.lo.begin(), right.lo.end());
            s.hi.insert(s.hi.end(), right.hi.begin(), right.hi.end());
            s.nodes[id].left = l;
            s.nodes[id].right = off;
        } else {
            const int32_t l = build_node(b, mid, depth + 1, par_depth, s);
            const int32_t r = build_node(mid, e, depth + 1, par_depth, s);
            s.nodes[id].left = l;
            s.nodes[id].right = r;
        }
        return id;
    }

    // Lower bound on dist(q, y) for y in the node's box, same operation order as dist().
    double boxdist(int32_t node, const double* q) const {
        const double* L = &lo[size_t(node) * d];
        const double* H = &hi[size_t(node) * d];
        double s = 0.0;
        for (int t = 0; t < d; ++t) {
            double g = 0.0;
            if (q[t] < L[t]) g = L[t] - q[t];
            else if (q[t] > H[t]) g = q[t] - H[t];
            s += g * g;
        }
        return std::sqrt(s);
    }

    // Calls leaf(begin, end) for every leaf that may hold a point within r of q and
    // whose id range intersects [idlo, idhi].
    template <class F>
    void visit(const double* q, double r, int32_t idlo, int32_t idhi, F&& leaf) const {
        int32_t stack[128];
        int sp = 0;
        stack[sp++] = 0;
        while (sp) {
            const Node& nd = nodes[stack[--sp]];
            if (nd.maxid < idlo || nd.minid > idhi) continue;
            int32_t id = int32_t(&nd - nodes.data());
            if (boxdist(id, q) > r) continue;
            if (nd.left < 0) {
                leaf(nd.begin, nd.end);
            } else {
                stack[sp++] = nd.right;
                stack[sp++] = nd.left;
            }
        }
    }

    // Ordering update around q.  ub[node] bounds m[j] from above for every
    // unselected point j of the node (m only decreases, so a stale bound stays
    // valid).  A node is entered only if its box may hold a point closer to q
    // than that bound -- the only points whose m can change.  leaf(begin, end)
    // updates a leaf and returns the exact maximum of m over its unselected
    // points (-inf if none), which becomes the leaf's bound; inner nodes take
    // the maximum of their children.
    template <class F>
    double relax(int32_t id, const double* q, std::vector<double>& ub, F& leaf) const {
        if (!(boxdist(id, q) < ub[size_t(id)])) return ub[size_t(id)];
        const Node& nd = nodes[size_t(id)];
        const double u = nd.left < 0 ? leaf(nd.begin, nd.end)
                                     : std::max(relax(nd.left, q, ub, leaf), relax(nd.right, q, ub, leaf));
        ub[size_t(id)] = u;
        return u;
    }
};

// Indexed 4-ary max-heap on (key descending, id ascending), keys stored inline:
// a level of a sift reads one 64-byte group of children instead of chasing ids
// into the key array (a cache miss per comparison on large inputs).  The order
// is strict and total, so the sequence of pops is that of any correct heap.
// pos[slot] (caller-owned) locates a slot's entry; heaps over disjoint slot sets
// may share one pos array.
struct MaxHeap {
    struct Entry {
        double key;
        int32_t id;   // original index: breaks ties
        int32_t slot; // caller's slot of the entry (pos is indexed by it)
    };
    std::vector<Entry> store;
    Entry* h = nullptr;  // h[0] is the root; children of i are 4i+1 .. 4i+4
    int32_t* pos = nullptr;
    int64_t size = 0;

    static bool greater(const Entry& a, const Entry& b) { return a.key > b.key || (a.key == b.key && a.id < b.id); }
    void init(const std::vector<Entry>& entries, int32_t* posv) {
        const int64_t n = int64_t(entries.size());
        // element 1 on a 64-byte boundary, so every group of 4 children shares one line
        store.resize(size_t(n) + 8);
        const uintptr_t base = reinterpret_cast<uintptr_t>(store.data());
        const uintptr_t want = ((base + 16 + 63) & ~uintptr_t(63)) - 16;
        h = reinterpret_cast<Entry*>(want);
        pos = posv;
        for (int64_t i = 0; i < n; ++i) {
            h[i] = entries[size_t(i)];
            pos[size_t(h[i].slot)] = int32_t(i);
        }
        size = n;
        for (int64_t i = (n - 2) / 4; i >= 0; --i) sift_down(i);
    }
    void sift_down(int64_t i) {
        const Entry v = h[i];
        for (;;) {
            const int64_t c = 4 * i + 1;
            if (c >= size) break;
            const int64_t ce = std::min<int64_t>(c + 4, size);
            int64_t best = c;
            for (int64_t k = c + 1; k < ce; ++k)
                if (greater(h[k], h[best])) best = k;
            if (!greater(h[best], v)) break;
            h[i] = h[best];
            pos[size_t(h[i].slot)] = int32_t(i);
            i = best;
        }
        h[i] = v;
        pos[size_t(v.slot)] = int32_t(i);
    }
    void sift_up(int64_t i) {
        const Entry v = h[i];
        while (i > 0) {
            const int64_t up = (i - 1) / 4;
            if (!greater(v, h[up])) break;
            h[i] = h[up];
            pos[size_t(h[i].slot)] = int32_t(i);
            i = up;
        }
        h[i] = v;
        pos[size_t(v.slot)] = int32_t(i);
    }
    // the key of slot s decreased to `key`
    void decrease(int32_t s, double key) {
        const int64_t i = pos[size_t(s)];
        h[i].key = key;
        sift_down(i);
    }
    // removes the maximum; returns its slot
    int32_t pop() {
        const int32_t top = h[0].slot;
        --size;
        if (size > 0) {
            h[0] = h[size];
            pos[size_t(h[0].slot)] = 0;
            sift_down(0);
        }
        pos[size_t(top)] = -1;
        return top;
    }
    // puts back an entry popped from this heap
    void push(const Entry& e) {
        h[size] = e;
        sift_up(size++);
    }
};

// Reusable barrier for a fixed team of threads: spins briefly, then sleeps, so
// that teams of concurrent analyses (a server's) do not burn each other's cores.
class TeamBarrier {
    static constexpr int kSpins = 1 << 10;

public:
    explicit TeamBarrier(int n) : n_(n) {}
    void wait() {
        const int g = gen_.load(std::memory_order_acquire);
        if (count_.fetch_add(1, std::memory_order_acq_rel) == n_ - 1) {
            count_.store(0, std::memory_order_relaxed);
            {
                std::lock_guard<std::mutex> lk(mu_);
                gen_.fetch_add(1, std::memory_order_release);
            }
            cv_.notify_all();
            return;
        }
        for (int spins = 0; spins < kSpins; ++spins) {
            if (gen_.load(std::memory_order_acquire) != g) return;
            __builtin_ia32_pause();
        }
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return gen_.load(std::memory_order_acquire) != g; });
    }

private:
    int n_;
    std::atomic<int> count_{0};
    std::atomic<int> gen_{0};
    std::mutex mu_;
    std::condition_variable cv_;
};

// The ordering runs in batches on several threads (at most kOrderThreads)
// only from kParallelOrderMin points and when the analysis is given at least
// kOrderThreadsMin threads: the batches add work (conflict checks, merging the
// heaps' candidates) that shortens one analysis but costs throughput when
// concurrent analyses share the cores, and a batch waits for its slowest
// thread four times, so more threads gain little.
constexpr int64_t kParallelOrderMin = 16384;
constexpr int kOrderThreads = 4;
constexpr int kOrderThreadsMin = 8;

// The exact greedy maximin ordering on several threads: the same output as the
// one-thread loop in maximin_order, by this argument.  Candidates leave the
// heaps in the one-thread pop order (current distance m descending, index
// ascending).  The first is the next point.  A later candidate c is the next
// point after the candidates already taken in the batch if no taken point a has
// dist(a, c) < m[c]: c's distance is then unchanged by them, every other
// point's distance only fell, so c still leads that order.  The first
// candidate that fails ends the batch and, with those after it, returns to its
// heap.  A batch's updates m[j] = min(m[j], dist(x_j, x_a)) commute, so the
// threads apply them at once, each to the points of the k-d subtrees it owns
// (with its own heap over them), and the comparisons that decide the output
// are those of the one-thread loop.
void maximin_parallel(const KDTree& tree, const std::vector<double>& xt, int64_t n, int32_t d, int nthreads,
                      int32_t* perm, double* l) {
    const int P = nthreads;
    // subtrees to share out: a frontier of at least 8 per thread
    std::vector<int32_t> parts{0};
    for (bool grew = true; grew && int64_t(parts.size()) < 8 * int64_t(P);) {
        grew = false;
        std::vector<int32_t> next;
        for (int32_t q : parts) {
            const auto& nd = tree.nodes[size_t(q)];
            if (nd.left >= 0) {
                next.push_back(nd.left);
                next.push_back(nd.right);
                grew = true;
            } else {
                next.push_back(q);
            }
        }
        parts.swap(next);
    }
    std::vector<std::vector<int32_t>> mine(static_cast<size_t>(P));
    for (size_t q = 0; q < parts.size(); ++q) mine[q % size_t(P)].push_back(parts[q]);
    std::vector<double> m(size_t(n), std::numeric_limits<double>::infinity());
    std::vector<char> sel(size_t(n), 0);
    std::vector<int32_t> pos(size_t(n), -1);
    std::vector<MaxHeap> heaps(static_cast<size_t>(P));
    for (int t = 0; t < P; ++t) {
        std::vector<MaxHeap::Entry> e;
        for (int32_t q : mine[size_t(t)])
            for (int32_t s = tree.nodes[size_t(q)].begin; s < tree.nodes[size_t(q)].end; ++s)
                e.push_back(MaxHeap::Entry{std::numeric_limits<double>::infinity(), tree.idx[size_t(s)], s});
        heaps[size_t(t)].init(e, pos.data());
    }
    std::vector<double> ub(tree.nodes.size(), std::numeric_limits<double>::infinity());

    std::vector<MaxHeap::Entry> cand;
    std::vector<int32_t> owner;
    std::vector<int32_t> taken;
    std::atomic<int64_t> conflict{0};
    int64_t k = 0, batch = 16;
    bool done = false;
    TeamBarrier bar(P);
    auto team = [&](int t) {
        MaxHeap& heap = heaps[size_t(t)];
        const double* xi = nullptr;
        auto leaf_update = [&](int32_t b, int32_t e) {
            double u = -std::numeric_limits<double>::infinity();
            for (int32_t s = b; s < e; ++s) {
                if (sel[size_t(s)]) continue;
                const double dj = dist(xt.data() + size_t(s) * d, xi, d);
                if (dj < m[size_t(s)]) {
                    m[size_t(s)] = dj;
                    heap.decrease(s, dj);
                }
                u = std::max(u, m[size_t(s)]);
            }
            return u;
        };
        for (;;) {
            if (t == 0) {  // the next candidates, in pop order
                cand.clear();
                owner.clear();
                while (int64_t(cand.size()) < batch) {
                    int best = -1;
                    for (int q = 0; q < P; ++q)
                        if (heaps[size_t(q)].size > 0 &&
                            (best < 0 || MaxHeap::greater(heaps[size_t(q)].h[0], heaps[size_t(best)].h[0])))
                            best = q;
                    if (best < 0) break;
                    cand.push_back(heaps[size_t(best)].h[0]);
                    owner.push_back(best);
                    heaps[size_t(best)].pop();
                }
                done = cand.empty();
                conflict.store(int64_t(cand.size()), std::memory_order_relaxed);
            }
            bar.wait();
            if (done) break;
            // first candidate within its own distance of an earlier one
            const int64_t nc = int64_t(cand.size());
            for (int64_t j = 1 + t; j < nc; j += P) {
                if (j >= conflict.load(std::memory_order_relaxed)) break;
                const double* xj = xt.data() + size_t(cand[size_t(j)].slot) * d;
                for (int64_t i = 0; i < j; ++i)
                    if (dist(xt.data() + size_t(cand[size_t(i)].slot) * d, xj, d) < cand[size_t(j)].key) {
                        int64_t cur = conflict.load(std::memory_order_relaxed);
                        while (j < cur && !conflict.compare_exchange_weak(cur, j, std::memory_order_relaxed)) {
                        }
                        break;
                    }
            }
            bar.wait();
            if (t == 0) {
                const int64_t J = conflict.load(std::memory_order_relaxed);
                taken.clear();
                for (int64_t i = 0; i < J; ++i) {
                    const int32_t s = cand[size_t(i)].slot;
                    perm[k] = tree.idx[size_t(s)];
                    l[k] = cand[size_t(i)].key;
                    ++k;
                    sel[size_t(s)] = 1;
                    taken.push_back(s);
                }
                for (int64_t i = J; i < nc; ++i) heaps[size_t(owner[size_t(i)])].push(cand[size_t(i)]);
                batch = std::min<int64_t>(512, std::max<int64_t>(16, 2 * J + 16));
            }
            bar.wait();
            // the batch's updates, on this thread's subtrees
            for (int32_t s : taken) {
                xi = xt.data() + size_t(s) * d;
                for (int32_t q : mine[size_t(t)]) tree.relax(q, xi, ub, leaf_update);
            }
            bar.wait();
        }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < P; ++t) pool.emplace_back(team, t);
    team(0);
    for (auto& th : pool) th.join();
}

}  // namespace

void maximin_order(const double* x, int64_t n, int32_t d, int nthreads, int32_t* perm, double* l) {
    KDTree tree;
    tree.build(x, n, d, resolve_threads(nthreads));
    // The working arrays are laid out in tree order (slot t holds point tree.idx[t]),
    // so that scanning a leaf reads contiguous memory.
    std::vector<double> xt(size_t(n) * d);
    for (int64_t t = 0; t < n; ++t)
        std::copy(x + size_t(tree.idx[t]) * d, x + size_t(tree.idx[t] + 1) * d, xt.begin() + size_t(t) * d);
    nthreads = resolve_threads(nthreads);
    if (nthreads >= kOrderThreadsMin && n >= kParallelOrderMin) {
        maximin_parallel(tree, xt, n, d, std::min(nthreads, kOrderThreads), perm, l);
        return;
    }
    std::vector<double> m(static_cast<size_t>(n), std::numeric_limits<double>::infinity());
    std::vector<char> sel(static_cast<size_t>(n), 0);
    std::vector<int32_t> pos(static_cast<size_t>(n), -1);
    MaxHeap heap;
    {
        std::vector<MaxHeap::Entry> e(static_cast<size_t>(n));
        for (int64_t t = 0; t < n; ++t) e[size_t(t)] = MaxHeap::Entry{m[size_t(t)], tree.idx[size_t(t)], int32_t(t)};
        heap.init(e, pos.data());
    }
    std::vector<double> ub(tree.nodes.size(), std::numeric_limits<double>::infinity());
    const double* xi = nullptr;
    auto leaf_update = [&](int32_t b, int32_t e) {
        double u = -std::numeric_limits<double>::infinity();
        for (int32_t t = b; t < e; ++t) {
            if (sel[size_t(t)]) continue;
            const double dj = dist(xt.data() + size_t(t) * d, xi, d);
            if (dj < m[size_t(t)]) {
                m[size_t(t)] = dj;
                heap.decrease(t, dj);
            }
            u = std::max(u, m[size_t(t)]);
        }
        return u;
    };
    for (int64_t k = 0; k < n; ++k) {
        const int32_t t = heap.pop();
        perm[k] = tree.idx[size_t(t)];
        l[k] = m[size_t(t)];
        sel[size_t(t)] = 1;
        xi = xt.data() + size_t(t) * d;
        // Only points with dist(x_j, x_i) < m[j] change.
        tree.relax(0, xi, ub, leaf_update);
    }
}

namespace {

void csr_from_csc(Plan& p, int nthreads) {
    // Rows start on multiples of kRowAlign entries and are padded with INT32_MAX.
    // Threads own balanced ranges of columns; a row's entries from thread t are
    // placed after those of threads t' < t, so rows stay sorted by column.
    const int64_t n = p.n, nnz = p.nnz();
    const int T = std::max(1, std::min<int>(nthreads, int(std::max<int64_t>(1, nnz / 4096))));
    std::vector<int64_t> cut(static_cast<size_t>(T + 1), n);
    cut[0] = 0;
    for (int t = 1; t < T; ++t)
        cut[t] = std::lower_bound(p.colptr.begin(), p.colptr.end(), nnz * t / T) - p.colptr.begin();
    for (int t = 1; t <= T; ++t) cut[t] = std::max(cut[t], cut[t - 1]);
    std::vector<std::vector<int64_t>> base(static_cast<size_t>(T));
    parallel_for(T, T, 1, [&](int64_t t0, int64_t t1, int) {
        for (int64_t t = t0; t < t1; ++t) {
            std::vector<int64_t>& c = base[size_t(t)];
            c.assign(size_t(n), 0);
            for (int64_t e = p.colptr[cut[t]]; e < p.colptr[cut[t + 1]]; ++e) c[size_t(p.rowidx[e])]++;
        }
    });
    std::vector<int64_t> len(static_cast<size_t>(n), 0);
    parallel_for(T, n, 1 << 16, [&](int64_t k0, int64_t k1, int) {
        for (int64_t k = k0; k < k1; ++k) {
            int64_t acc = 0;
            for (int t = 0; t < T; ++t) {
                const int64_t c = base[size_t(t)][size_t(k)];
                base[size_t(t)][size_t(k)] = acc;  // offset of thread t's entries inside row k
                acc += c;
            }
            len[size_t(k)] = acc;
        }
    });
    p.rowptr.assign(size_t(n + 1), 0);
    p.rowend.resize(size_t(n));
    p.max_row = 0;
    for (int64_t k = 0; k < n; ++k) {
        p.rowend[k] = p.rowptr[k] + len[k];
        p.rowptr[k + 1] = p.rowptr[k] + (len[k] + kRowAlign - 1) / kRowAlign * kRowAlign;
        p.max_row = std::max(p.max_row, len[k]);
    }
    p.colidx.assign(size_t(p.rowptr[n]), INT32_MAX);
    p.csc2csr.resize(size_t(nnz));
    parallel_for(T, T, 1, [&](int64_t t0, int64_t t1, int) {
        for (int64_t t = t0; t < t1; ++t) {
            std::vector<int64_t>& off = base[size_t(t)];
            for (int64_t j = cut[t]; j < cut[t + 1]; ++j)
                for (int64_t e = p.colptr[j]; e < p.colptr[j + 1]; ++e) {
                    const int64_t k = p.rowidx[e];
                    const int64_t q = p.rowptr[k] + off[size_t(k)]++;
                    p.colidx[size_t(q)] = int32_t(j);
                    p.csc2csr[size_t(e)] = uint32_t(q);
                }
        }
    });
    encode_row_deltas(p, nthreads);
}

}  // namespace

namespace {

// dist(a,b) <= R with the canonical expression.  The running sum of squares is
// the canonical one and only grows, so once it exceeds R2 -- an upper bound on
// every s with sqrt(s) <= R after rounding -- the point cannot be within R.
inline bool within(const double* a, const double* b, int d, double R, double R2) {
    double s = 0.0;
    for (int t = 0; t < d; ++t) {
        double df = a[t] - b[t];
        s += df * df;
        if (s > R2) return false;
    }
    return std::sqrt(s) <= R;
}

inline double r2_bound(double R) { return R * R * (1.0 + 1e-12) + 1e-300; }

// Runs scan(i, buf) for i in [0, n) on parallel chunks; scan appends item i's
// values to buf.  The values are concatenated in order of i into vals, with
// offsets ptr (n + 1).  One pass: each chunk's values stay in the buffer of the
// thread that produced them until the final copy.
template <class Scan>
void collect(int nthreads, int64_t n, Scan&& scan, std::vector<int64_t>& ptr, std::vector<int32_t>& vals) {
    // The first items (the coarsest columns, whose balls cover most points) get a
    // chunk each so that no thread is left with all the heavy ones.
    constexpr int64_t kHeavy = 4096, kChunkItems = 64;
    const int64_t nheavy = std::min(n, kHeavy);
    const int64_t nchunks = nheavy + (n - nheavy + kChunkItems - 1) / kChunkItems;
    auto chunk_begin = [&](int64_t c) { return c < nheavy ? c : nheavy + (c - nheavy) * kChunkItems; };
    nthreads = std::max(1, nthreads);
    std::vector<std::vector<int32_t>> bufs(static_cast<size_t>(nthreads));
    std::vector<int32_t> chunk_thread(static_cast<size_t>(nchunks));
    std::vector<int64_t> chunk_off(static_cast<size_t>(nchunks));
    std::vector<int64_t> cnt(static_cast<size_t>(n), 0);
    parallel_for(nthreads, nchunks, 1, [&](int64_t c0, int64_t c1, int tid) {
        std::vector<int32_t>& buf = bufs[size_t(tid)];
        for (int64_t c = c0; c < c1; ++c) {
            chunk_thread[size_t(c)] = tid;
            chunk_off[size_t(c)] = int64_t(buf.size());
            const int64_t i1 = std::min(n, chunk_begin(c + 1));
            for (int64_t i = chunk_begin(c); i < i1; ++i) {
                const size_t before = buf.size();
                scan(i, buf);
                cnt[size_t(i)] = int64_t(buf.size() - before);
            }
        }
    });
    ptr.assign(size_t(n + 1), 0);
    for (int64_t i = 0; i < n; ++i) ptr[size_t(i + 1)] = ptr[size_t(i)] + cnt[size_t(i)];
    vals.resize(size_t(ptr[size_t(n)]));
    parallel_for(nthreads, nchunks, 16, [&](int64_t c0, int64_t c1, int) {
        for (int64_t c = c0; c < c1; ++c) {
            const int64_t i0 = chunk_begin(c), i1 = std::min(n, chunk_begin(c + 1));
            const int32_t* src = bufs[size_t(chunk_thread[size_t(c)])].data() + chunk_off[size_t(c)];
            std::copy(src, src + (ptr[size_t(i1)] - ptr[size_t(i0)]), vals.data() + ptr[size_t(i0)]);
        }
    });
}

}  // namespace

void encode_row_deltas(Plan& p, int nthreads) {
    nthreads = resolve_threads(nthreads);
    const int64_t n = p.n;
    const int64_t lim = p.delta_limit;
    p.cdelta.assign(size_t(p.nnz_rows()), 0);
    std::vector<uint32_t> cnt(static_cast<size_t>(n), 0);
    parallel_for(nthreads, n, 1 << 12, [&](int64_t k0, int64_t k1, int) {
        for (int64_t k = k0; k < k1; ++k) {
            int64_t prev = -1;
            uint32_t c = 0;
            for (int64_t q = p.rowptr[k]; q < p.rowend[k]; ++q) {
                const int64_t g = int64_t(p.colidx[size_t(q)]) - prev;
                if (g >= lim) ++c;
                else p.cdelta[size_t(q)] = uint16_t(g);
                prev = p.colidx[size_t(q)];
            }
            cnt[size_t(k)] = c;
        }
    });
    p.escptr.assign(size_t(n + 1), 0);
    for (int64_t k = 0; k < n; ++k) p.escptr[size_t(k + 1)] = p.escptr[size_t(k)] + cnt[size_t(k)];
    p.esc.assign(size_t(p.escptr[size_t(n)]), 0);
    parallel_for(nthreads, n, 1 << 12, [&](int64_t k0, int64_t k1, int) {
        for (int64_t k = k0; k < k1; ++k) {
            int64_t prev = -1;
            uint32_t w = p.escptr[size_t(k)];
            for (int64_t q = p.rowptr[k]; q < p.rowend[k]; ++q) {
                if (int64_t(p.colidx[size_t(q)]) - prev >= lim) p.esc[size_t(w++)] = p.colidx[size_t(q)];
                prev = p.colidx[size_t(q)];
            }
        }
    });
}

void build_pattern(Plan& p, int nthreads) {
    nthreads = resolve_threads(nthreads);
    const int64_t n = p.n;
    const int d = p.d;
    const double* xh = p.xh.data();
    KDTree tree;
    tree.build(xh, n, d, nthreads);
    p.spatial = tree.idx;  // k-d tree leaf order: positions grouped by region
    // points copied into tree order, so that scanning a leaf reads contiguous memory
    const std::vector<int32_t>& idt = tree.idx;
    std::vector<double> xt(size_t(n) * d);
    parallel_for(nthreads, n, 1 << 14, [&](int64_t t0, int64_t t1, int) {
        for (int64_t t = t0; t < t1; ++t)
            std::copy(xh + size_t(idt[size_t(t)]) * d, xh + size_t(idt[size_t(t)] + 1) * d, xt.begin() + size_t(t) * d);
    });

    if (p.rule == KC_RULE_MAX) {
        // column b: the diagonal, then rows a > b with dist(x_a, x_b) <= rho * max(l_a, l_b) = rho * l_b
        collect(nthreads, n, [&](int64_t b, std::vector<int32_t>& out) {
            const double* xb = xh + size_t(b) * d;
            const double R = p.rho * p.l[size_t(b)], R2 = r2_bound(R);
            out.push_back(int32_t(b));
            const size_t first = out.size();
            tree.visit(xb, R, int32_t(b + 1), int32_t(n - 1), [&](int32_t s, int32_t e) {
                for (int32_t t = s; t < e; ++t) {
                    const int32_t a = idt[size_t(t)];
                    if (a > b && within(xt.data() + size_t(t) * d, xb, d, R, R2)) out.push_back(a);
                }
            });
            std::sort(out.begin() + first, out.end());
        }, p.colptr, p.rowidx);
    } else {
        // row a: columns b < a with dist(x_a, x_b) <= rho * min(l_a, l_b) = rho * l_a
        std::vector<int64_t> rp;
        std::vector<int32_t> cols;
        collect(nthreads, n, [&](int64_t a, std::vector<int32_t>& out) {
            const double* xa = xh + size_t(a) * d;
            const double R = p.rho * p.l[size_t(a)], R2 = r2_bound(R);
            tree.visit(xa, R, 0, int32_t(a - 1), [&](int32_t s, int32_t e) {
                for (int32_t t = s; t < e; ++t) {
                    const int32_t b = idt[size_t(t)];
                    if (b < a && within(xa, xt.data() + size_t(t) * d, d, R, R2)) out.push_back(b);
                }
            });
        }, rp, cols);
        // transpose rows into CSC columns (diagonal first, rows ascending)
        std::vector<int64_t> cnt(static_cast<size_t>(n), 1);
        for (int32_t b : cols) cnt[size_t(b)]++;
        p.colptr.assign(size_t(n + 1), 0);
        for (int64_t b = 0; b < n; ++b) p.colptr[b + 1] = p.colptr[b] + cnt[b];
        if (p.colptr[n] >= (int64_t(1) << 32)) return;
        p.rowidx.resize(size_t(p.colptr[n]));
        std::vector<int64_t> fill(p.colptr.begin(), p.colptr.end() - 1);
        for (int64_t b = 0; b < n; ++b) p.rowidx[size_t(fill[b]++)] = int32_t(b);
        for (int64_t a = 0; a < n; ++a)
            for (int64_t q = rp[a]; q < rp[a + 1]; ++q) p.rowidx[size_t(fill[cols[q]]++)] = int32_t(a);
    }
    if (p.colptr[n] >= (int64_t(1) << 32)) return;  // caller reports KC_ERANGE
    p.max_col = 0;
    for (int64_t b = 0; b < n; ++b) p.max_col = std::max(p.max_col, p.colptr[b + 1] - p.colptr[b]);
    csr_from_csc(p, nthreads);
}

void build_schedule(Plan& p, int nthreads) {
    (void)nthreads;
    const int64_t n = p.n;
    // forward levels: column j after every parent i in row j
    p.level.assign(size_t(n), 0);
    for (int64_t j = 0; j < n; ++j) {
        int32_t lj = p.level[j] + 1;
        for (int64_t e = p.colptr[j] + 1; e < p.colptr[j + 1]; ++e) {
            int32_t k = p.rowidx[e];
            if (p.level[k] < lj) p.level[k] = lj;
        }
    }
    int32_t nl = 0;
    for (int64_t j = 0; j < n; ++j) nl = std::max(nl, p.level[j] + 1);
    p.nlevels = nl;
    std::vector<int64_t> loff(static_cast<size_t>(nl + 1), 0), uoff(size_t(nl + 1), 0);
    for (int64_t j = 0; j < n; ++j) {
        loff[size_t(p.level[j]) + 1]++;
        uoff[size_t(p.level[j]) + 1] += (p.colptr[j + 1] - p.colptr[j] + 63) / 64;
    }
    for (int32_t v = 0; v < nl; ++v) {
        loff[v + 1] += loff[v];
        uoff[v + 1] += uoff[v];
    }
    p.fwd_off = loff;
    p.unit_off = uoff;
    p.fwd_rows.resize(size_t(n));
    p.units.resize(size_t(uoff[nl]));
    {
        std::vector<int64_t> lf(loff.begin(), loff.end() - 1), uf(uoff.begin(), uoff.end() - 1);
        // within a level, columns follow the k-d tree leaf order, so that
        // consecutive work units touch nearby points and the same rows of L
        for (int64_t t = 0; t < n; ++t) {
            const int32_t j = p.spatial[size_t(t)];
            int32_t v = p.level[j];
            p.fwd_rows[size_t(lf[v]++)] = int32_t(j);
            int64_t len = p.colptr[j + 1] - p.colptr[j];
            for (int64_t c = 0; c < len; c += 64) p.units[size_t(uf[v]++)] = Unit{int32_t(j), int32_t(c)};
        }
    }
    // reverse levels: column j after every k > j in column j
    std::vector<int32_t> rl(static_cast<size_t>(n), 0);
    int32_t nrl = 0;
    for (int64_t j = n - 1; j >= 0; --j) {
        int32_t v = 0;
        for (int64_t e = p.colptr[j] + 1; e < p.colptr[j + 1]; ++e) v = std::max(v, rl[size_t(p.rowidx[e])] + 1);
        rl[size_t(j)] = v;
        nrl = std::max(nrl, v + 1);
    }
    p.nrlevels = nrl;
    p.bwd_off.assign(size_t(nrl + 1), 0);
    for (int64_t j = 0; j < n; ++j) p.bwd_off[size_t(rl[j]) + 1]++;
    for (int32_t v = 0; v < nrl; ++v) p.bwd_off[v + 1] += p.bwd_off[v];
    p.bwd_cols.resize(size_t(n));
    std::vector<int64_t> bf(p.bwd_off.begin(), p.bwd_off.end() - 1);
    // within a level, columns follow the k-d tree leaf order (as the forward
    // rows do), so that neighbouring work touches the same solution rows
    for (int64_t t = 0; t < n; ++t) {
        const int32_t j = p.spatial[size_t(t)];
        p.bwd_cols[size_t(bf[rl[j]]++)] = j;
    }
}

}  // namespace kc

namespace kc {

// The union of independent problems is one problem whose pattern is block
// diagonal: positions, rows and columns of instance i are shifted by the
// number of points before it, and its DAG levels are merged level by level
// with the other instances' (columns of different instances never depend on
// each other), so one launch per level serves every instance at that depth.
void merge_plans(const std::vector<Plan>& parts, Plan& out) {
    const int32_t ni = int32_t(parts.size());
    out = Plan();
    out.ninst = ni;
    out.d = parts.empty() ? 0 : parts[0].d;
    out.rho = parts.empty() ? 0.0 : parts[0].rho;
    out.rule = parts.empty() ? 0 : parts[0].rule;
    out.inst_off.assign(size_t(ni + 1), 0);
    int64_t nnz = 0, nnzr = 0;
    for (int32_t i = 0; i < ni; ++i) {
        out.inst_off[i + 1] = out.inst_off[i] + parts[i].n;
        nnz += parts[i].nnz();
        nnzr += parts[i].nnz_rows();
        out.nlevels = std::max(out.nlevels, parts[i].nlevels);
        out.nrlevels = std::max(out.nrlevels, parts[i].nrlevels);
        out.max_col = std::max(out.max_col, parts[i].max_col);
        out.max_row = std::max(out.max_row, parts[i].max_row);
    }
    const int64_t n = out.inst_off[ni];
    out.n = n;
    out.perm.resize(size_t(n));
    out.l.resize(size_t(n));
    out.xh.resize(size_t(n) * out.d);
    out.spatial.resize(size_t(n));
    out.inst.resize(size_t(n));
    out.level.resize(size_t(n));
    out.colptr.assign(size_t(n + 1), 0);
    out.rowidx.resize(size_t(nnz));
    out.rowptr.assign(size_t(n + 1), 0);
    out.rowend.resize(size_t(n));
    out.colidx.resize(size_t(nnzr));
    out.csc2csr.resize(size_t(nnz));
    int64_t e0 = 0, q0 = 0;
    for (int32_t i = 0; i < ni; ++i) {
        const Plan& p = parts[i];
        const int64_t b = out.inst_off[i];
        for (int64_t k = 0; k < p.n; ++k) {
            out.perm[b + k] = int32_t(b + p.perm[k]);
            out.l[b + k] = p.l[k];
            out.spatial[b + k] = int32_t(b + p.spatial[k]);
            out.inst[b + k] = i;
            out.level[b + k] = p.level[k];
            out.colptr[b + k + 1] = e0 + p.colptr[k + 1];
            out.rowptr[b + k + 1] = q0 + p.rowptr[k + 1];
            out.rowend[b + k] = q0 + p.rowend[k];
        }
        std::copy(p.xh.begin(), p.xh.end(), out.xh.begin() + b * out.d);
        for (int64_t e = 0; e < p.nnz(); ++e) {
            out.rowidx[e0 + e] = int32_t(b + p.rowidx[e]);
            out.csc2csr[e0 + e] = uint32_t(q0 + p.csc2csr[e]);
        }
        for (int64_t q = 0; q < p.nnz_rows(); ++q)
            out.colidx[q0 + q] = p.colidx[q] == INT32_MAX ? INT32_MAX : int32_t(b + p.colidx[q]);
        e0 += p.nnz();
        q0 += p.nnz_rows();
    }
    encode_row_deltas(out, 0);
    // level-major merge of units and forward rows
    out.unit_off.assign(size_t(out.nlevels + 1), 0);
    out.fwd_off.assign(size_t(out.nlevels + 1), 0);
    for (int32_t v = 0; v < out.nlevels; ++v) {
        int64_t u = 0, r = 0;
        for (const Plan& p : parts)
            if (v < p.nlevels) {
                u += p.unit_off[v + 1] - p.unit_off[v];
                r += p.fwd_off[v + 1] - p.fwd_off[v];
            }
        out.unit_off[v + 1] = out.unit_off[v] + u;
        out.fwd_off[v + 1] = out.fwd_off[v] + r;
    }
    out.units.resize(size_t(out.unit_off[out.nlevels]));
    out.fwd_rows.resize(size_t(n));
    for (int32_t v = 0; v < out.nlevels; ++v) {
        int64_t u = out.unit_off[v], r = out.fwd_off[v];
        for (int32_t i = 0; i < ni; ++i) {
            const Plan& p = parts[i];
            if (v >= p.nlevels) continue;
            const int32_t b = int32_t(out.inst_off[i]);
            for (int64_t t = p.unit_off[v]; t < p.unit_off[v + 1]; ++t)
                out.units[size_t(u++)] = Unit{b + p.units[t].col, p.units[t].first};
            for (int64_t t = p.fwd_off[v]; t < p.fwd_off[v + 1]; ++t) out.fwd_rows[size_t(r++)] = b + p.fwd_rows[t];
        }
    }
    out.bwd_off.assign(size_t(out.nrlevels + 1), 0);
    for (int32_t v = 0; v < out.nrlevels; ++v) {
        int64_t c = 0;
        for (const Plan& p : parts)
            if (v < p.nrlevels) c += p.bwd_off[v + 1] - p.bwd_off[v];
        out.bwd_off[v + 1] = out.bwd_off[v] + c;
    }
    out.bwd_cols.resize(size_t(n));
    for (int32_t v = 0; v < out.nrlevels; ++v) {
        int64_t c = out.bwd_off[v];
        for (int32_t i = 0; i < ni; ++i) {
            const Plan& p = parts[i];
            if (v >= p.nrlevels) continue;
            const int32_t b = int32_t(out.inst_off[i]);
            for (int64_t t = p.bwd_off[v]; t < p.bwd_off[v + 1]; ++t) out.bwd_cols[size_t(c++)] = b + p.bwd_cols[t];
        }
    }
    for (const Plan& p : parts) {
        out.t_order += p.t_order;
        out.t_pattern += p.t_pattern;
        out.t_schedule += p.t_schedule;
    }
}

}  // namespace kc

namespace kc {

// Supernodal ordering and sparsity pattern, after the construction in the
// paper's stability analysis (Section 5, supernodal multicolor construction):
//  * aggregation: greedily in maximin order, an unassigned point k starts a
//    supernode and claims every later unassigned point a of the same scale
//    (l_a >= l_k / 2) within 0.5 * rho * l_k;
//  * ordering: supernodes by their first point, members consecutively in
//    maximin order (the colouring is not needed: the level schedule of the
//    elimination DAG provides the parallelism);
//  * pattern: supernodes A and B are adjacent when some member pair is in the
//    pattern S_rho; the new pattern contains every member pair of adjacent
//    supernodes (the block closure), so the factor's nonzeros form dense blocks.
void supernodal_transform(Plan& p, int nthreads) {
    nthreads = resolve_threads(nthreads);
    const int64_t n = p.n;
    const int d = p.d;
    const double* xh = p.xh.data();
    // 1. aggregation
    std::vector<int32_t> node(static_cast<size_t>(n), -1);
    std::vector<int64_t> leader;
    {
        KDTree tree;
        tree.build(xh, n, d);
        for (int64_t k = 0; k < n; ++k) {
            if (node[size_t(k)] >= 0) continue;
            const int32_t s = int32_t(leader.size());
            leader.push_back(k);
            node[size_t(k)] = s;
            const double R = 0.5 * p.rho * p.l[size_t(k)], R2 = r2_bound(R), lmin = 0.5 * p.l[size_t(k)];
            const double* xk = xh + size_t(k) * d;
            tree.visit(xk, R, int32_t(k + 1), int32_t(n - 1), [&](int32_t b, int32_t e) {
                for (int32_t t = b; t < e; ++t) {
                    const int32_t a = tree.idx[t];
                    if (a > k && node[size_t(a)] < 0 && p.l[size_t(a)] >= lmin && within(xh + size_t(a) * d, xk, d, R, R2))
                        node[size_t(a)] = s;
                }
            });
        }
    }
    const int64_t ns = int64_t(leader.size());
    // 2. new order: supernodes in order of their first point, members in maximin order
    std::vector<int64_t> sptr(static_cast<size_t>(ns + 1), 0);
    for (int64_t k = 0; k < n; ++k) sptr[size_t(node[size_t(k)]) + 1]++;
    for (int64_t s = 0; s < ns; ++s) sptr[size_t(s + 1)] += sptr[size_t(s)];
    std::vector<int64_t> newpos(static_cast<size_t>(n));
    std::vector<int32_t> oldpos(static_cast<size_t>(n));
    {
        std::vector<int64_t> fill(sptr.begin(), sptr.end() - 1);
        for (int64_t k = 0; k < n; ++k) {
            const int64_t q = fill[size_t(node[size_t(k)])]++;
            newpos[size_t(k)] = q;
            oldpos[size_t(q)] = int32_t(k);
        }
    }
    // 3. supernode adjacency (symmetric), kept for the larger supernode index of each pair
    std::vector<std::vector<int32_t>> adj(static_cast<size_t>(ns));
    parallel_for(nthreads, ns, 64, [&](int64_t s0, int64_t s1, int) {
        std::vector<int64_t> stamp;
        for (int64_t s = s0; s < s1; ++s) {
            std::vector<int32_t>& out = adj[size_t(s)];
            auto add = [&](int32_t t) {
                if (t >= s) out.push_back(t);
            };
            for (int64_t q = sptr[size_t(s)]; q < sptr[size_t(s + 1)]; ++q) {
                const int64_t c = oldpos[size_t(q)];
                for (int64_t e = p.colptr[c]; e < p.colptr[c + 1]; ++e) add(node[size_t(p.rowidx[e])]);
                for (int64_t e = p.rowptr[c]; e < p.rowend[c]; ++e) add(node[size_t(p.colidx[e])]);
            }
            std::sort(out.begin(), out.end());
            out.erase(std::unique(out.begin(), out.end()), out.end());
        }
    });
    // 4. block-closed pattern in the new positions
    std::vector<int64_t> colptr(static_cast<size_t>(n + 1), 0);
    for (int64_t s = 0; s < ns; ++s) {
        int64_t below = 0;
        for (int32_t t : adj[size_t(s)])
            if (t > s) below += sptr[size_t(t + 1)] - sptr[size_t(t)];
        for (int64_t q = sptr[size_t(s)]; q < sptr[size_t(s + 1)]; ++q) colptr[size_t(q + 1)] = below + (sptr[size_t(s + 1)] - q);
    }
    for (int64_t q = 0; q < n; ++q) colptr[size_t(q + 1)] += colptr[size_t(q)];
    std::vector<int32_t> rowidx(static_cast<size_t>(colptr[static_cast<size_t>(n)]));
    parallel_for(nthreads, ns, 64, [&](int64_t s0, int64_t s1, int) {
        for (int64_t s = s0; s < s1; ++s)
            for (int64_t q = sptr[size_t(s)]; q < sptr[size_t(s + 1)]; ++q) {
                int64_t w = colptr[size_t(q)];
                for (int64_t r = q; r < sptr[size_t(s + 1)]; ++r) rowidx[size_t(w++)] = int32_t(r);
                for (int32_t t : adj[size_t(s)])
                    if (t > s)
                        for (int64_t r = sptr[size_t(t)]; r < sptr[size_t(t + 1)]; ++r) rowidx[size_t(w++)] = int32_t(r);
            }
    });
    // 5. replace ordering, points and pattern
    std::vector<int32_t> perm(static_cast<size_t>(n));
    std::vector<double> l(static_cast<size_t>(n)), xn(size_t(n) * d);
    for (int64_t q = 0; q < n; ++q) {
        const int64_t k = oldpos[size_t(q)];
        perm[size_t(q)] = p.perm[size_t(k)];
        l[size_t(q)] = p.l[size_t(k)];
        for (int t = 0; t < d; ++t) xn[size_t(q) * d + t] = xh[size_t(k) * d + t];
    }
    for (auto& v : p.spatial) v = int32_t(newpos[size_t(v)]);
    p.perm.swap(perm);
    p.l.swap(l);
    p.xh.swap(xn);
    p.colptr.swap(colptr);
    p.rowidx.swap(rowidx);
    p.snode_ptr.swap(sptr);
    if (p.nnz() >= (int64_t(1) << 32)) return;
    p.max_col = 0;
    for (int64_t b = 0; b < n; ++b) p.max_col = std::max(p.max_col, p.colptr[b + 1] - p.colptr[b]);
    csr_from_csc(p, nthreads);
}

}  // namespace kc
