// Host side of the batched contingency PCG library: the C ABI declared in
// include/gpcg.h, argument checks, the host preparation passes (matrix
// assembly, ILU(0), integer topology pass, triangular-solve scheduling) and
// the device context.
#include "../../include/gpcg.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <map>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "gpcg_internal.h"

namespace {

thread_local std::string g_last_error;

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(int code, const std::string &msg) { throw Error(code, msg); }

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) fail(GPCG_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class F>
int guarded(F &&f) {
    try {
        g_last_error.clear();
        f();
        return GPCG_OK;
    } catch (const Error &e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return GPCG_E_NOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return GPCG_E_ARG;
    } catch (...) {
        g_last_error = "unknown error";
        return GPCG_E_ARG;
    }
}

// ---------------------------------------------------------------------------
// CSR checks
void check_csr(const gpcg_csr *M, const char *name, int n_expect) {
    if (!M) fail(GPCG_E_ARG, std::string(name) + " is NULL");
    if (M->n != n_expect) fail(GPCG_E_ARG, std::string(name) + " has the wrong size");
    if (M->n < 0 || M->nnz < 0 || (M->n > 0 && (!M->rowptr || (M->nnz > 0 && (!M->col || !M->val)))))
        fail(GPCG_E_ARG, std::string(name) + ": missing arrays");
    if (M->n == 0) return;
    if (M->rowptr[0] != 0 || M->rowptr[M->n] != M->nnz) fail(GPCG_E_PATTERN, std::string(name) + ": bad rowptr");
    for (int i = 0; i < M->n; ++i) {
        if (M->rowptr[i + 1] < M->rowptr[i]) fail(GPCG_E_PATTERN, std::string(name) + ": rowptr decreases");
        for (int e = M->rowptr[i]; e < M->rowptr[i + 1]; ++e) {
            const int j = M->col[e];
            if (j < 0 || j >= M->n) fail(GPCG_E_PATTERN, std::string(name) + ": column out of range");
            if (e > M->rowptr[i] && M->col[e - 1] >= j) fail(GPCG_E_PATTERN, std::string(name) + ": unsorted row");
            if (!std::isfinite(M->val[e])) fail(GPCG_E_ARG, std::string(name) + ": non-finite value");
        }
    }
}

void check_branches(int n_bus, int m, const int32_t *from, const int32_t *to, const double *x) {
    if (n_bus < 1 || m < 0) fail(GPCG_E_ARG, "need n_bus >= 1 and m >= 0");
    if (m > 0 && (!from || !to)) fail(GPCG_E_ARG, "branch endpoints are NULL");
    for (int e = 0; e < m; ++e) {
        if (from[e] < 0 || from[e] >= n_bus || to[e] < 0 || to[e] >= n_bus || from[e] == to[e])
            fail(GPCG_E_ARG, "branch endpoint out of range or a self-loop");
        if (x && !(x[e] > 0.0 && std::isfinite(x[e]))) fail(GPCG_E_ARG, "branch reactance must be positive and finite");
    }
}

// ---------------------------------------------------------------------------
// Correctly rounded sum of doubles: the exact sum is carried as a list of
// non-overlapping partials (Shewchuk, "Adaptive precision floating-point
// arithmetic and fast robust geometric predicates", 1997), which are then
// added from the largest down; a final check settles the half-way case, where
// the rounding of the leading pair has to be decided by the sign of the rest.
double exact_sum(const std::vector<double> &terms) {
    std::vector<double> part;
    for (double x : terms) {
        size_t k = 0;
        for (double y : part) {
            if (std::fabs(x) < std::fabs(y)) std::swap(x, y);
            const double hi = x + y;
            const double lo = y - (hi - x);
            if (lo != 0.0) part[k++] = lo;
            x = hi;
        }
        part.resize(k);
        part.push_back(x);
    }
    if (part.empty()) return 0.0;
    size_t n = part.size() - 1;
    double hi = part[n], lo = 0.0;
    while (n > 0) {
        const double x = hi, y = part[--n];
        hi = x + y;
        lo = y - (hi - x);
        if (lo != 0.0) break;
    }
    if (n > 0 && ((lo < 0.0 && part[n - 1] < 0.0) || (lo > 0.0 && part[n - 1] > 0.0))) {
        const double y = 2.0 * lo, x = hi + y;
        if (y == x - hi) hi = x;
    }
    return hi;
}

// ---------------------------------------------------------------------------
// Reduced susceptance matrix (slack = bus 0 dropped).  Every entry is the
// exact sum of its terms (each branch's rounded 1 / x, the shunt) rounded
// once, so the matrix does not depend on the order of the branch table.
int assemble(int n_bus, int m, const int32_t *from, const int32_t *to, const double *x, const double *shunt,
             std::vector<int32_t> &rowptr, std::vector<int32_t> &col, std::vector<double> &val) {
    const int nr = n_bus - 1;
    // per reduced row: (column, term) pairs, the diagonal's terms included
    std::vector<std::vector<std::pair<int, double>>> rows(nr);
    for (int e = 0; e < m; ++e) {
        const double b = 1.0 / x[e];
        const int f = from[e] - 1, t = to[e] - 1;
        if (f >= 0) rows[f].push_back({f, b});
        if (t >= 0) rows[t].push_back({t, b});
        if (f >= 0 && t >= 0) {
            rows[f].push_back({t, -b});
            rows[t].push_back({f, -b});
        }
    }
    rowptr.assign(nr + 1, 0);
    col.clear();
    val.clear();
    std::vector<double> terms;
    for (int i = 0; i < nr; ++i) {
        auto &r = rows[i];
        if (shunt) r.push_back({i, shunt[i + 1]});
        r.push_back({i, 0.0});  // every row keeps its diagonal entry
        std::stable_sort(r.begin(), r.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
        for (size_t k = 0; k < r.size();) {
            size_t k1 = k;
            terms.clear();
            while (k1 < r.size() && r[k1].first == r[k].first) terms.push_back(r[k1++].second);
            col.push_back(r[k].first);
            val.push_back(exact_sum(terms));  // parallel branches add up
            k = k1;
        }
        rowptr[i + 1] = (int32_t)col.size();
    }
    return (int)col.size();
}

// Reverse Cuthill-McKee order of the buses other than the slack (the slack
// and its branches leave the reduced system).  Every connected piece starts
// at its bus of least degree (ties by bus number); a breadth-first search
// appends each bus's unvisited neighbours by increasing degree (ties by bus
// number), and the whole sequence is reversed.  (A pseudo-peripheral start
// gave a slightly smaller bandwidth but longer triangular dependency chains
// and more PCG iterations on the synthetic grids.)  perm[k] is the bus of
// reduced row k.
std::vector<int32_t> rcm_order(int n_bus, int m, const int32_t *from, const int32_t *to) {
    std::vector<std::vector<int>> adj(n_bus);
    for (int e = 0; e < m; ++e) {
        if (from[e] == 0 || to[e] == 0) continue;
        adj[from[e]].push_back(to[e]);
        adj[to[e]].push_back(from[e]);
    }
    std::vector<int> deg(n_bus, 0);
    for (int v = 1; v < n_bus; ++v) {
        auto &a = adj[v];
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
        deg[v] = (int)a.size();
    }
    auto lighter = [&](int x, int y) { return deg[x] != deg[y] ? deg[x] < deg[y] : x < y; };
    for (int v = 1; v < n_bus; ++v) std::sort(adj[v].begin(), adj[v].end(), lighter);
    std::vector<char> seen(n_bus, 0), mark(n_bus, 0);
    std::vector<int> piece, seq;
    seq.reserve(n_bus - 1);
    for (int s0 = 1; s0 < n_bus; ++s0) {
        if (mark[s0]) continue;
        // the piece of s0 and its lightest bus
        piece.assign(1, s0);
        seen[s0] = 1;
        for (size_t t = 0; t < piece.size(); ++t)
            for (int w : adj[piece[t]])
                if (!seen[w]) {
                    seen[w] = 1;
                    piece.push_back(w);
                }
        const int root = *std::min_element(piece.begin(), piece.end(), lighter);
        size_t head = seq.size();
        seq.push_back(root);
        mark[root] = 1;
        while (head < seq.size()) {
            const int v = seq[head++];
            for (int w : adj[v])
                if (!mark[w]) {
                    mark[w] = 1;
                    seq.push_back(w);
                }
        }
    }
    std::reverse(seq.begin(), seq.end());
    return std::vector<int32_t>(seq.begin(), seq.end());
}

// Check that perm holds every bus 1 .. n_bus - 1 once; returns inv with
// inv[perm[k]] = k + 1 (the internal bus) and inv[0] = 0.
std::vector<int32_t> invert_perm(int n_bus, const int32_t *perm) {
    std::vector<int32_t> inv(n_bus, -1);
    inv[0] = 0;
    for (int k = 0; k < n_bus - 1; ++k) {
        const int b = perm[k];
        if (b < 1 || b >= n_bus || inv[b] >= 0) fail(GPCG_E_ARG, "perm must hold each bus 1 .. n_bus - 1 once");
        inv[b] = k + 1;
    }
    return inv;
}

// Zero-fill incomplete LU, IKJ order (Saad, Alg. 10.4), with a dense
// column-to-position map of the current row.
void ilu0(const gpcg_csr &A, std::vector<double> &F, std::vector<int> &diagpos) {
    const int n = A.n;
    F.assign(A.val, A.val + A.nnz);
    diagpos.assign(n, -1);
    for (int i = 0; i < n; ++i)
        for (int e = A.rowptr[i]; e < A.rowptr[i + 1]; ++e)
            if (A.col[e] == i) diagpos[i] = e;
    for (int i = 0; i < n; ++i)
        if (diagpos[i] < 0) fail(GPCG_E_PATTERN, "row " + std::to_string(i) + " has no diagonal entry");
    std::vector<int> pos(n, -1);
    for (int i = 0; i < n; ++i) {
        for (int e = A.rowptr[i]; e < A.rowptr[i + 1]; ++e) pos[A.col[e]] = e;
        for (int e = A.rowptr[i]; e < A.rowptr[i + 1]; ++e) {
            const int k = A.col[e];
            if (k >= i) break;
            const double piv = F[diagpos[k]];
            if (piv == 0.0) fail(GPCG_E_PIVOT, "zero pivot at row " + std::to_string(k));
            F[e] /= piv;
            const double lik = F[e];
            for (int q = diagpos[k] + 1; q < A.rowptr[k + 1]; ++q) {
                const int pj = pos[A.col[q]];
                if (pj >= 0) F[pj] -= lik * F[q];
            }
        }
        for (int e = A.rowptr[i]; e < A.rowptr[i + 1]; ++e) pos[A.col[e]] = -1;
    }
}

// Iterative DFS from the slack with low-link values; the tree edge into v is
// remembered by branch id so a parallel branch counts as a back edge.
struct Topology {
    std::vector<uint8_t> is_bridge;
    std::vector<int32_t> pre, sub, lo, hi;
    int n_bridges = 0;
};

Topology topology(int n_bus, int m, const int32_t *from, const int32_t *to) {
    Topology T;
    std::vector<int> adj_ptr(n_bus + 1, 0), adj(2 * (size_t)m), adj_e(2 * (size_t)m);
    for (int e = 0; e < m; ++e) {
        adj_ptr[from[e] + 1]++;
        adj_ptr[to[e] + 1]++;
    }
    for (int v = 0; v < n_bus; ++v) adj_ptr[v + 1] += adj_ptr[v];
    std::vector<int> fill(adj_ptr.begin(), adj_ptr.end() - 1);
    for (int e = 0; e < m; ++e) {
        adj[fill[from[e]]] = to[e];
        adj_e[fill[from[e]]++] = e;
        adj[fill[to[e]]] = from[e];
        adj_e[fill[to[e]]++] = e;
    }
    T.pre.assign(n_bus, -1);
    T.sub.assign(n_bus, 1);
    T.is_bridge.assign(m, 0);
    T.lo.assign(m, 0);
    T.hi.assign(m, 0);
    std::vector<int> low(n_bus), parent_edge(n_bus, -1), it(n_bus), stack;
    int counter = 0;
    if (n_bus > 0) {
        stack.push_back(0);
        T.pre[0] = low[0] = counter++;
        it[0] = adj_ptr[0];
        while (!stack.empty()) {
            const int v = stack.back();
            if (it[v] < adj_ptr[v + 1]) {
                const int k = it[v]++;
                const int w = adj[k], e = adj_e[k];
                if (e == parent_edge[v]) continue;
                if (T.pre[w] < 0) {
                    T.pre[w] = low[w] = counter++;
                    parent_edge[w] = e;
                    it[w] = adj_ptr[w];
                    stack.push_back(w);
                } else {
                    low[v] = std::min(low[v], T.pre[w]);
                }
            } else {
                stack.pop_back();
                if (!stack.empty()) {
                    const int u = stack.back();
                    low[u] = std::min(low[u], low[v]);
                    T.sub[u] += T.sub[v];
                    if (low[v] > T.pre[u]) {
                        const int e = parent_edge[v];
                        T.is_bridge[e] = 1;
                        T.lo[e] = T.pre[v];
                        T.hi[e] = T.pre[v] + T.sub[v];
                        T.n_bridges++;
                    }
                }
            }
        }
    }
    if (counter != n_bus) fail(GPCG_E_ARG, "the grid is not connected");
    return T;
}

// ---------------------------------------------------------------------------
// Triangular-solve schedule.  deps[i] lists the rows row i needs, all of them
// "earlier" (smaller index for the forward solve; the backward solve is run
// on mirrored indices).  Each step takes up to R ready rows, scanning from
// the lowest unfinished row over a window of `look` rows, so the rows in
// flight stay close together and a small LDS ring can hold every value that
// is still to be read.
struct Schedule {
    int R = 1, steps = 0, ring = 1;
    std::vector<int32_t> rows;  // steps x R, -1 = idle
};

Schedule build_schedule(int n, int R, int look, const std::vector<std::vector<int>> &deps) {
    Schedule S;
    S.R = R;
    std::vector<int> done_step(n, -1);
    int lowest = 0, processed = 0, step = 0;
    std::vector<int> pick;
    while (processed < n) {
        pick.clear();
        const int end = std::min(n, lowest + std::max(look, R));
        for (int i = lowest; i < end && (int)pick.size() < R; ++i) {
            if (done_step[i] >= 0) continue;
            bool ready = true;
            for (int j : deps[i])
                if (done_step[j] < 0) {
                    ready = false;
                    break;
                }
            if (ready) pick.push_back(i);
        }
        if (pick.empty()) fail(GPCG_E_PATTERN, "triangular factor has a dependency cycle");
        for (int i : pick) done_step[i] = step;
        for (int k = 0; k < R; ++k) S.rows.push_back(k < (int)pick.size() ? pick[k] : -1);
        processed += (int)pick.size();
        while (lowest < n && done_step[lowest] >= 0) ++lowest;
        ++step;
    }
    S.steps = step;
    return S;
}

// ---------------------------------------------------------------------------
template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    void alloc(size_t count) {
        if (p) {
            (void)hipFree(p);
            p = nullptr;
        }
        n = count;
        if (count == 0) return;
        if (hipMalloc((void **)&p, count * sizeof(T)) != hipSuccess) {
            p = nullptr;
            n = 0;
            fail(GPCG_E_NOMEM, "device allocation failed");
        }
    }
    void upload(const T *src, size_t count, hipStream_t st) {
        alloc(count);
        if (count) hip_check(hipMemcpyAsync(p, src, count * sizeof(T), hipMemcpyHostToDevice, st), "upload");
    }
};

// Host copy of a CSR matrix (the context keeps A, L and strict-upper U).
struct CsrH {
    std::vector<int32_t> rowptr, col;
    std::vector<double> val;
    int len(int i) const { return rowptr[i + 1] - rowptr[i]; }
};

// A sweep program in host memory (see gpcg::Program).
struct HostProg {
    int steps = 0, ring = 1;
    std::vector<int32_t> rec;  // 4 per (step, slot)
    std::vector<int32_t> ent;  // 3 per (step, entry, slot), chunk-major (see gpcg::Program); staged: blocks
};

// One slot of a step before packing.
struct Slot {
    int row = -1;    // row finished here (-1 none)
    int la = -1;     // product: look-ahead row whose direction is updated
    bool cont = false;
    int seg_begin = 0, seg_end = 0;  // entries [begin, end) of the row `src`
    int src = -1;                    // row whose entries this slot multiplies
};

using Steps = std::vector<std::vector<Slot>>;

// Split every row of a step list into segments of at most K entries: the
// continuation segments go to extra steps placed right before the step,
// in the same slot.  Look-ahead updates move to the first of those steps.
Steps expand(const Steps &in, int R, int K, const CsrH &T) {
    Steps out;
    for (const auto &st : in) {
        int extra = 0;
        for (const Slot &sl : st)
            if (sl.row >= 0) extra = std::max(extra, (std::max(T.len(sl.row), 1) + K - 1) / K - 1);
        for (int c = 0; c <= extra; ++c) {
            std::vector<Slot> o(R);
            for (int k = 0; k < R; ++k) {
                const Slot &sl = st[k];
                if (c == 0) o[k].la = sl.la;
                if (sl.row < 0) continue;
                const int nseg = std::max(1, (T.len(sl.row) + K - 1) / K);
                const int first = extra - (nseg - 1);  // step of the row's first segment
                if (c < first) continue;
                const int seg = c - first;
                o[k].src = sl.row;
                o[k].seg_begin = seg * K;
                o[k].seg_end = std::min(T.len(sl.row), seg * K + K);
                if (c == extra)
                    o[k].row = sl.row;
                else
                    o[k].cont = true;
            }
            out.push_back(std::move(o));
        }
    }
    return out;
}

// Smallest power-of-two ring that keeps every value a step reads: each step
// first writes its look-ahead rows (product), then reads the columns of its
// entries, then writes the rows it finishes (triangular solves).
int ring_needed(const Steps &st, const CsrH &T, bool tri, int max_ring) {
    for (int W = 1; W <= max_ring; W <<= 1) {
        std::vector<int> owner(W, -1);
        bool ok = true;
        for (const auto &step : st) {
            for (const Slot &sl : step)
                if (sl.la >= 0) owner[sl.la & (W - 1)] = sl.la;
            for (size_t a = 0; a < step.size() && ok; ++a)
                for (size_t b = 0; b < a && ok; ++b) {
                    if (step[a].la >= 0 && step[b].la >= 0 && ((step[a].la ^ step[b].la) & (W - 1)) == 0) ok = false;
                    if (tri && step[a].row >= 0 && step[b].row >= 0 && ((step[a].row ^ step[b].row) & (W - 1)) == 0)
                        ok = false;
                }
            for (const Slot &sl : step) {
                if (sl.src < 0) continue;
                for (int e = T.rowptr[sl.src] + sl.seg_begin; e < T.rowptr[sl.src] + sl.seg_end; ++e)
                    if (owner[T.col[e] & (W - 1)] != T.col[e]) ok = false;
                if (!tri && sl.row >= 0 && owner[sl.row & (W - 1)] != sl.row) ok = false;  // p_i read for p'q
            }
            if (tri)
                for (const Slot &sl : step)
                    if (sl.row >= 0) owner[sl.row & (W - 1)] = sl.row;
            if (!ok) break;
        }
        if (ok) return W;
    }
    return -1;
}

// Pack an expanded step list for the kernel (see gpcg::Program).
// Whether the factors have the form U = D L^T, D = diag(U), to rounding
// (each strictly upper U_ij within 1e-12 relative of U_ii L_ji, and the
// other way round): then M = L U is symmetric and, with r zero on islanded
// rows, r'z = r' (L U)^-1 r = y' D^-1 y for y = L^-1 r (Section III.A's
// inner product, summed in the forward sweep).  The ILU(0) of a symmetric
// matrix and the Jacobi pair have this form.
bool factors_symmetric(const CsrH &L, const CsrH &Us, const std::vector<double> &invdiag) {
    const int n = (int)L.rowptr.size() - 1;
    auto at = [](const CsrH &T, int row, int col) {
        const int32_t *b = T.col.data() + T.rowptr[row], *t = T.col.data() + T.rowptr[row + 1];
        const int32_t *f = std::lower_bound(b, t, col);
        return (f != t && *f == col) ? T.val[f - T.col.data()] : 0.0;
    };
    auto close = [](double u, double v) { return std::fabs(u - v) <= 1e-12 * std::max(std::fabs(u), std::fabs(v)); };
    for (int i = 0; i < n; ++i)
        for (int e = Us.rowptr[i]; e < Us.rowptr[i + 1]; ++e)  // U_ij against U_ii L_ji
            if (!close(Us.val[e], at(L, Us.col[e], i) / invdiag[i])) return false;
    for (int j = 0; j < n; ++j)
        for (int e = L.rowptr[j]; e < L.rowptr[j + 1]; ++e) {  // L_ji against U_ij / U_ii
            const int i = L.col[e];
            if (!close(at(Us, i, j), L.val[e] / invdiag[i])) return false;
        }
    return true;
}

HostProg pack(const Steps &st, int R, int S, int ring, int K, const CsrH &T, bool tri,
              const std::vector<double> *invdiag, const std::vector<int32_t> &prerow) {
    HostProg H;
    H.ring = ring;
    H.steps = (int)st.size();
    const int zero = ring * S * 8, trash = (ring + 1) * S * 8;
    Steps all = st;  // plus idle steps that the kernel's prefetch may read past the end
    all.insert(all.end(), gpcg::kPadSteps, std::vector<Slot>(R));
    const int nr = (int)T.rowptr.size() - 1;  // idle slots name the scratch row n_r
    for (const auto &step : all) {
        for (int k = 0; k < R; ++k) {
            const Slot &sl = step[k];
            const int row = sl.row >= 0 ? sl.row : nr;
            const int aux = sl.cont ? 1 : (sl.row >= 0 ? 0 : -1);
            if (invdiag) {  // backward solve: packed record with 1 / U_ii
                const int slot = sl.row >= 0 ? (sl.row & (ring - 1)) : ring + 1;  // trash row when idle
                const int pre = sl.row >= 0 ? prerow[sl.row] : gpcg::kBwdRowMask;
                const double dv = sl.row >= 0 ? (*invdiag)[sl.row] : 0.0;
                int32_t w[2];
                std::memcpy(w, &dv, sizeof dv);
                H.rec.push_back(row | (slot << gpcg::kBwdRowBits));
                H.rec.push_back(pre | ((aux + 1) << gpcg::kBwdRowBits));
                H.rec.push_back(w[0]);
                H.rec.push_back(w[1]);
                continue;
            }
            H.rec.push_back(row);
            H.rec.push_back(sl.row >= 0 ? (sl.row & (ring - 1)) * S * 8 : (tri ? trash : zero));
            if (tri) {
                H.rec.push_back(sl.row >= 0 ? prerow[sl.row] : -1);
                H.rec.push_back(aux);
            } else {
                H.rec.push_back(sl.cont ? -2 : (sl.row >= 0 ? prerow[sl.row] : -1));
                H.rec.push_back(sl.la >= 0 ? sl.la : nr);
            }
        }
        // per slot: K values (two to a 16-byte chunk), then K ring offsets
        // (four to a chunk); stored chunk-major, chunk c of slot k at
        // ((step, c), k)
        std::vector<int32_t> w((size_t)R * 3 * K);
        for (int k = 0; k < R; ++k) {
            const Slot &sl = step[k];
            int32_t *vals = &w[(size_t)k * 3 * K], *offs = vals + 2 * K;
            for (int j = 0; j < K; ++j) {
                double v = 0.0;
                int lds = zero;
                if (sl.src >= 0 && sl.seg_begin + j < sl.seg_end) {
                    const int e = T.rowptr[sl.src] + sl.seg_begin + j;
                    v = T.val[e];
                    lds = (T.col[e] & (ring - 1)) * S * 8;
                }
                std::memcpy(vals + 2 * j, &v, sizeof v);
                offs[j] = lds;
            }
        }
        for (int c = 0; c < 3 * K / 4; ++c)
            for (int k = 0; k < R; ++k)
                for (int t = 0; t < 4; ++t) H.ent.push_back(w[(size_t)k * 3 * K + c * 4 + t]);
    }
    if (gpcg::staged(S, K)) {
        // staged blocks: step s's entry chunks, then the records of step
        // s + ahead (the last, idle, padding step's past the end)
        const size_t n = all.size(), ent_step = (size_t)R * 3 * K, rec_step = (size_t)R * 4;
        const size_t ahead = (size_t)gpcg::stage_rec_ahead(tri);
        std::vector<int32_t> blocks;
        blocks.reserve(n * (ent_step + rec_step));
        for (size_t st_i = 0; st_i < n; ++st_i) {
            blocks.insert(blocks.end(), H.ent.begin() + st_i * ent_step, H.ent.begin() + (st_i + 1) * ent_step);
            const size_t r = std::min(st_i + ahead, n - 1);
            blocks.insert(blocks.end(), H.rec.begin() + r * rec_step, H.rec.begin() + (r + 1) * rec_step);
        }
        H.ent.swap(blocks);
    }
    return H;
}

// Step list of a triangular solve from its schedule (rows per step).
Steps tri_steps(const std::vector<int32_t> &sched, int R) {
    Steps st(sched.size() / R, std::vector<Slot>(R));
    for (size_t s = 0; s < st.size(); ++s)
        for (int k = 0; k < R; ++k) {
            const int row = sched[s * R + k];
            st[s][k].row = row;
            st[s][k].src = row;
            st[s][k].seg_begin = 0;
            st[s][k].seg_end = 0;  // set by expand()
        }
    return st;
}

// Step list of the product sweep: step c holds rows c R .. c R + R - 1 and
// updates the direction of rows (c + lead) R ..; `lead` prologue steps come
// first.
Steps prod_steps(int nr, int R, int lead) {
    const int chunks = (nr + R - 1) / R;
    Steps st;
    for (int c = -lead; c < chunks; ++c) {
        std::vector<Slot> step(R);
        for (int k = 0; k < R; ++k) {
            const int la = (c + lead) * R + k;
            step[k].la = (c + lead < chunks && la < nr) ? la : -1;
            const int row = c * R + k;
            step[k].row = (c >= 0 && row < nr) ? row : -1;
        }
        st.push_back(std::move(step));
    }
    return st;
}

struct DevProgram {
    int steps = 0, ring = 1;
    DevBuf<int32_t> rec, ent;
    void upload(const HostProg &H, hipStream_t st) {
        steps = H.steps;
        ring = H.ring;
        rec.upload(H.rec.data(), H.rec.size(), st);
        ent.upload(H.ent.data(), H.ent.size(), st);
    }
    gpcg::Program view() const {
        gpcg::Program g{};
        g.rec = (const int4 *)rec.p;
        g.ent = (const int4 *)ent.p;
        g.steps = steps;
        g.ring = ring;
        return g;
    }
};

struct DevSchedule {
    int R = 1;
    DevProgram f, b, p;
    int ring_max() const { return std::max(f.ring, std::max(b.ring, p.ring)); }
};

}  // namespace

struct gpcg_context {
    int device = 0;
    hipStream_t stream = nullptr;
    int n_bus = 0, m = 0, n_r = 0, kind = GPCG_KIND_BP, S = 64, look = 256, bandwidth = 0, zero_start = 0;
    int nnz_a = 0, nnz_l = 0, nnz_u = 0;
    DevBuf<int32_t> a_rowptr, a_col, l_rowptr, l_col, u_rowptr, u_col;
    DevBuf<double> a_val, l_val, u_val, u_invdiag;
    // the matrix side in internal buses (row i = internal bus i + 1); the
    // bus side (flows, overload, power flow) in the caller's numbering
    DevBuf<int32_t> br_from, br_to, pre_row, pre_bus, isl_lo, isl_hi;
    DevBuf<int32_t> cbr_from, cbr_to, cpre_bus, bus_map;  // bus_map: internal -> caller (none: identity)
    std::vector<int32_t> perm, inv;                       // row -> caller's bus, caller's bus -> internal (empty: identity)
    DevBuf<double> br_x, br_b, theta_b, rho_b, scal;
    DevBuf<double> ws, gfac, partial;
    DevBuf<int32_t> queue;               // the PCG launch's queue counter
    DevBuf<int32_t> hist_base, hist_cols;  // iterations of each outage (index c + 1) in the last solve of each mode
    bool rec_base = false, rec_cols = false;  // an ordered solve of that mode has recorded iterations
    DevBuf<unsigned long long> sweeps;   // iterations summed over the waves of the last launch
    int last_waves = 0;                  // waves of the last PCG launch
    int max_waves[7] = {0, 0, 0, 0, 0, 0, 0};  // wavefronts that fit the device at once, per log2(block)
    DevBuf<int32_t> inc_ptr, inc_br;  // branches at each bus
    DevBuf<double> ov_theta, ov_flows, ov_g, ov_lambda;  // overload-gradient workspace
    DevBuf<double> diag_bus;                             // diagonal of A by bus (slack 0), built on first use
    DevBuf<double> fd_rhs, fd_dx, fd_gfac;               // power-flow workspace
    DevBuf<int32_t> fd_nogen, fd_it, fd_st;
    int spmm_ch = 0, spmm_max_nnz = 0;  // chunk layout of A the stand-alone product reads
    DevBuf<double> c_val;
    DevBuf<int32_t> c_col, c_rp, c_pre;
    DevBuf<uint32_t> keys, keys_sorted;
    DevBuf<int32_t> iota, order, pos;
    DevBuf<char> sort_temp;
    std::vector<std::vector<int>> deps_f, deps_b;  // for schedule building
    CsrH hA, hL, hU;                               // A, L, strict upper of U
    std::vector<double> h_invdiag;
    bool sym_factors = false;  // U = D L^T to rounding (see factors_symmetric)
    std::vector<int32_t> h_prerow;
    // sweep programs per (block, look-ahead window), shared with the batches
    // that use them
    std::map<std::pair<int, int>, std::shared_ptr<DevSchedule>> scheds;
    Topology topo;
    std::vector<double> theta_b_host;
    int base_iters = 0;
    double base_resid = 0.0;
    bool timing = false, timed = false;
    int last_n_out = 0;
    bool last_ordered = false;
    const int32_t *last_order = nullptr;  // device order of the last batched solve (context or fixed scratch)
    hipEvent_t ev0 = nullptr, ev1 = nullptr;

    ~gpcg_context() {
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
    }

    // The sweep programs for block S_ with a triangular look-ahead window of
    // look_ rows (0: the context's), built once and kept.
    std::shared_ptr<DevSchedule> schedule_ptr(int S_, int look_ = 0) {
        if (look_ <= 0) look_ = look;
        std::shared_ptr<DevSchedule> &slot = scheds[{S_, look_}];
        if (!slot) slot = build_schedules(S_, look_);
        return slot;
    }
    DevSchedule &schedule_for(int S_, int look_ = 0) { return *schedule_ptr(S_, look_); }

    std::shared_ptr<DevSchedule> build_schedules(int S_, int look0) {
        const int R = gpcg::kWave / S_;
        auto D = std::make_shared<DevSchedule>();
        D->R = R;
        // ring rows + the zero row + the trash row must fit the LDS budget
        const int max_ring = std::max(1, gpcg::kLdsBudget / (int)(S_ * sizeof(double)) - 2);
        const int lead = (bandwidth + R - 1) / R;
        const Steps P = expand(prod_steps(n_r, R, lead), R, gpcg::kEntProd, hA);
        const int wp = ring_needed(P, hA, false, max_ring);
        if (wp < 0)
            fail(GPCG_E_UNSUPPORTED, "the matrix bandwidth needs a larger LDS ring than a wavefront may use; "
                                     "give a banded row order (gpcg_options.perm, e.g. from gpcg_rcm) or set "
                                     "gpcg_options.reorder, or use a smaller block");
        for (int look_try = look0;; look_try /= 2) {
            Schedule F = build_schedule(n_r, R, look_try, deps_f);
            Schedule B = build_schedule(n_r, R, look_try, deps_b);
            // the backward schedule was built on mirrored indices
            for (auto &v : B.rows)
                if (v >= 0) v = n_r - 1 - v;
            const Steps FS = expand(tri_steps(F.rows, R), R, gpcg::kEntTri, hL);
            const Steps BS = expand(tri_steps(B.rows, R), R, gpcg::kEntTri, hU);
            const int wf = ring_needed(FS, hL, true, std::min(max_ring, gpcg::kBwdMaxRing));
            const int wb = ring_needed(BS, hU, true, std::min(max_ring, gpcg::kBwdMaxRing));
            if (wf > 0 && wb > 0) {
                D->f.upload(pack(FS, R, S_, wf, gpcg::kEntTri, hL, true, &h_invdiag, h_prerow), stream);
                D->b.upload(pack(BS, R, S_, wb, gpcg::kEntTri, hU, true, &h_invdiag, h_prerow), stream);
                D->p.upload(pack(P, R, S_, wp, gpcg::kEntProd, hA, false, nullptr, h_prerow), stream);
                hip_check(hipStreamSynchronize(stream), "schedule upload");
                break;
            }
            if (look_try <= R)
                fail(GPCG_E_UNSUPPORTED, "the factors' bandwidth needs a larger LDS ring than a wavefront may use; "
                                         "give a banded row order (gpcg_options.perm, e.g. from gpcg_rcm) or set "
                                         "gpcg_options.reorder");
        }
        return D;
    }

    gpcg::PcgParams params(const DevSchedule &D, const int32_t *outages, int n_out, const double *rhs, double tol,
                           int max_iter, int32_t *iters, int32_t *status) {
        gpcg::PcgParams p{};
        p.n_r = n_r;
        p.n_bus = n_bus;
        p.m = m;
        p.kind = kind;
        p.bus_map = bus_map.p;
        p.fwd = D.f.view();
        p.bwd = D.b.view();
        p.prod = D.p.view();
        p.br_from = br_from.p;
        p.br_to = br_to.p;
        p.br_b = br_b.p;
        p.pre_row = pre_row.p;
        p.isl_lo = isl_lo.p;
        p.isl_hi = isl_hi.p;
        p.theta_b = theta_b.p;
        p.rho_b = rho_b.p;
        p.rhs = rhs;
        p.outages = outages;
        p.n_out = n_out;
        p.tol2 = tol * tol;
        p.max_iter = max_iter;
        p.queue = queue.p;
        p.sweeps = sweeps.p;
        p.sym = sym_factors ? 1 : 0;
        p.iters_out = iters;
        p.status_out = status;
        return p;
    }

    // Persistent wavefronts of a launch at block S_: one scenario at a time
    // for the plain form (S_ = 1), else as many as fit the device at once,
    // but no more than the scenarios need.
    int waves_for(int S_, int n_out, const DevSchedule &D) {
        if (S_ == 1) return 1;
        int lg = 0;
        while ((1 << lg) < S_) ++lg;
        if (!max_waves[lg]) {
            max_waves[lg] = gpcg::pcg_max_waves(S_, D.ring_max());
            if (max_waves[lg] <= 0) fail(GPCG_E_HIP, "occupancy query of the PCG kernel failed");
        }
        return std::max(1, std::min(max_waves[lg], (n_out + S_ - 1) / S_));
    }

    size_t ws_slot(int S_) const { return (size_t)gpcg::kVectors * gpcg::vec_stride(n_r, S_); }

    int internal_bus(int k) const { return inv.empty() ? k : inv[k]; }
};

namespace {

// Device memory one batched solve works in: the waves' vectors, the
// per-scenario re-dispatch factors and the buffers of the scenario ordering.
struct Work {
    int n_waves = 0;
    size_t ws_slot = 0;
    double *ws = nullptr, *gfac = nullptr;
    uint32_t *keys = nullptr, *keys_sorted = nullptr;
    int32_t *iota = nullptr, *order = nullptr, *pos = nullptr;
    void *temp = nullptr;
    size_t temp_bytes = 0;
};

bool needs_order(int S_, int n_out) { return S_ > 1 && n_out > S_; }

// The context's own workspace, grown on demand.
Work context_work(gpcg_context *h, int n_out, int S_, const DevSchedule &D) {
    Work w;
    w.n_waves = h->waves_for(S_, n_out, D);
    w.ws_slot = h->ws_slot(S_);
    if (h->ws.n < (size_t)w.n_waves * w.ws_slot) h->ws.alloc((size_t)w.n_waves * w.ws_slot);
    if (h->gfac.n < (size_t)std::max(n_out, 1)) h->gfac.alloc(std::max(n_out, 1));
    w.ws = h->ws.p;
    w.gfac = h->gfac.p;
    if (needs_order(S_, n_out)) {
        if (h->keys.n < (size_t)n_out) {
            h->keys.alloc(n_out);
            h->keys_sorted.alloc(n_out);
            h->iota.alloc(n_out);
            h->order.alloc(n_out);
            h->pos.alloc(n_out);
        }
        const size_t tb = gpcg::sort_temp_bytes(n_out);
        if (h->sort_temp.n < tb) h->sort_temp.alloc(tb);
        w.keys = h->keys.p;
        w.keys_sorted = h->keys_sorted.p;
        w.iota = h->iota.p;
        w.order = h->order.p;
        w.pos = h->pos.p;
        w.temp = h->sort_temp.p;
        w.temp_bytes = tb;
    }
    return w;
}

// The same buffers carved out of the library's fixed device scratch (no
// allocation): the per-scenario buffers first, then as many wave slots as
// the rest holds (at most what the launch would use).  Fails when not even
// one wave slot fits.
Work static_work(gpcg_context *h, int n_out, int S_, const DevSchedule &D) {
    void *base = nullptr;
    hip_check(gpcg::static_scratch(&base), "static scratch");
    size_t off = 0;
    auto take = [&](size_t bytes) {
        void *p = (char *)base + off;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    Work w;
    w.gfac = (double *)take((size_t)n_out * sizeof(double));
    if (needs_order(S_, n_out)) {
        w.keys = (uint32_t *)take((size_t)n_out * sizeof(uint32_t));
        w.keys_sorted = (uint32_t *)take((size_t)n_out * sizeof(uint32_t));
        w.iota = (int32_t *)take((size_t)n_out * sizeof(int32_t));
        w.order = (int32_t *)take((size_t)n_out * sizeof(int32_t));
        w.pos = (int32_t *)take((size_t)n_out * sizeof(int32_t));
        w.temp_bytes = gpcg::sort_temp_bytes(n_out);
        w.temp = take(w.temp_bytes);
    }
    w.ws_slot = h->ws_slot(S_);
    const size_t slot_bytes = w.ws_slot * sizeof(double);
    const size_t room = off < gpcg::kStaticScratchBytes ? gpcg::kStaticScratchBytes - off : 0;
    const int fit = (int)std::min<size_t>(room / slot_bytes, (size_t)1 << 30);
    if (fit < 1)
        fail(GPCG_E_UNSUPPORTED, "the solve needs more than the " + std::to_string(gpcg::kStaticScratchBytes >> 20) +
                                     " MiB of the fixed scratch (" + std::to_string((off + slot_bytes) >> 20) +
                                     " MiB for one wavefront); solve fewer outages per call");
    w.n_waves = std::min(fit, h->waves_for(S_, n_out, D));
    w.ws = (double *)take((size_t)w.n_waves * slot_bytes);
    return w;
}

}  // namespace

namespace {

// Whether the PCG sweeps stream their vectors (the kernel's non-temporal
// form) for a workspace of ws_doubles doubles: only where the waves' vectors
// exceed the 256 MB Infinity Cache, which otherwise keeps them between
// sweeps (on the 2,000-bus grid, 179 MB of vectors, the streamed form took
// twice as long; on the 10,000-bus grid, 4.3 GB, it was 3.7 % faster).
bool streams_vectors(size_t ws_doubles) {
    constexpr size_t kInfinityCacheBytes = (size_t)256 << 20;
    return ws_doubles * sizeof(double) > kInfinityCacheBytes;
}

void run_solve(gpcg_context *h, int S_, int n_out, const int32_t *outages, const double *rhs, double tol,
               int max_iter, double *x_out, double *flows_out, int32_t *iters_out, int32_t *status_out,
               uint8_t *island_out, double *resid_out, const double *rhs_cols = nullptr, int rhs_ld = 0,
               bool fixed_scratch = false) {
    if (!h) fail(GPCG_E_ARG, "context is NULL");
    if (n_out < 0) fail(GPCG_E_ARG, "n_out < 0");
    if (n_out == 0) return;
    if (!outages || !(rhs || rhs_cols) || !x_out || !iters_out || !status_out)
        fail(GPCG_E_ARG, "a required pointer is NULL");
    if (rhs_cols && rhs_ld < h->n_bus) fail(GPCG_E_ARG, "ld must be >= n_bus");
    if (rhs_cols && flows_out) fail(GPCG_E_ARG, "flows are not formed for per-scenario right-hand sides");
    if (max_iter < 1) fail(GPCG_E_ARG, "max_iter must be >= 1");
    if (!(tol >= 0.0) || !std::isfinite(tol)) fail(GPCG_E_ARG, "tol must be finite and >= 0");
    if (flows_out && h->kind != GPCG_KIND_BP) fail(GPCG_E_ARG, "flows are only defined for a B' context");
    hip_check(hipSetDevice(h->device), "hipSetDevice");
    if (fixed_scratch && S_ != h->S) fail(GPCG_E_ARG, "the fixed-scratch solve runs at the context's block");
    DevSchedule &D = h->schedule_for(S_);  // built at setup for the context's block
    const Work w = fixed_scratch ? static_work(h, n_out, S_, D) : context_work(h, n_out, S_, D);
    // residual of the base state for this right-hand side, in double-double
    if (!rhs_cols)
        hip_check(gpcg::launch_base_residual(h->n_r, h->a_rowptr.p, h->a_col.p, h->a_val.p, h->theta_b.p, rhs,
                                             h->bus_map.p, h->rho_b.p, h->stream),
                  "base residual");
    gpcg::PcgParams p = h->params(D, outages, n_out, rhs, tol, max_iter, iters_out, status_out);
    p.ws = w.ws;
    p.ws_slot = w.ws_slot;
    p.gfac_out = w.gfac;
    p.x_out = x_out;
    p.rhs_cols = rhs_cols;
    p.rhs_ld = rhs_ld;
    p.zero_start = (!rhs_cols && h->zero_start) ? 1 : 0;
    p.add_base = (!rhs_cols && !h->zero_start) ? 1 : 0;
    int32_t *hist = rhs_cols ? h->hist_cols.p : h->hist_base.p;
    if (needs_order(S_, n_out)) {
        // the queue hands out the scenarios of most expected work first
        hip_check(gpcg::launch_order(n_out, outages, h->m, h->br_from.p, h->br_to.p, h->br_b.p, h->isl_lo.p,
                                     h->isl_hi.p, h->theta_b.p, hist, w.keys, w.keys_sorted, w.iota, w.order, w.pos,
                                     w.temp, w.temp_bytes, h->stream),
                  "scenario ordering");
        p.order = w.order;
    }
    h->last_order = p.order;
    h->last_n_out = n_out;
    h->last_ordered = p.order != nullptr;
    h->last_waves = w.n_waves;
    // a queue ranked by recorded iterations leaves few columns idle, and
    // vectors larger than the Infinity Cache are not kept by it: the sweeps
    // then stream their vectors (non-temporal hint)
    bool &recorded = rhs_cols ? h->rec_cols : h->rec_base;
    const bool streamed = p.order != nullptr && recorded && streams_vectors((size_t)w.n_waves * w.ws_slot);
    if (h->timing) hip_check(hipEventRecord(h->ev0, h->stream), "event");
    hip_check(gpcg::launch_pcg(p, S_, w.n_waves, D.ring_max(), streamed, h->stream), "pcg launch");
    if (needs_order(S_, n_out)) {
        hip_check(gpcg::launch_record_iters(n_out, outages, h->m, iters_out, hist, h->stream), "iteration records");
        recorded = true;
    }
    if (h->timing) {
        hip_check(hipEventRecord(h->ev1, h->stream), "event");
        h->timed = true;
    }
    gpcg::OutParams o{};
    o.n_r = h->n_r;
    o.n_bus = h->n_bus;
    o.m = h->m;
    o.kind = h->kind;
    o.n_out = n_out;
    o.bus_map = h->bus_map.p;
    o.cbr_from = h->cbr_from.p;
    o.cbr_to = h->cbr_to.p;
    o.a_rowptr = h->a_rowptr.p;
    o.a_col = h->a_col.p;
    o.a_val = h->a_val.p;
    o.br_from = h->br_from.p;
    o.br_to = h->br_to.p;
    o.br_x = h->br_x.p;
    o.br_b = h->br_b.p;
    o.pre_bus = h->pre_bus.p;
    o.isl_lo = h->isl_lo.p;
    o.isl_hi = h->isl_hi.p;
    o.theta_b = h->theta_b.p;
    o.rhs = rhs;
    o.rhs_cols = rhs_cols;
    o.rhs_ld = rhs_ld;
    o.add_base = (!rhs_cols && !h->zero_start) ? 1 : 0;
    o.outages = outages;
    o.status = status_out;
    o.gfac = w.gfac;
    o.x_out = x_out;
    o.flows_out = flows_out;
    o.resid_out = resid_out;
    o.island_out = island_out;
    hip_check(gpcg::launch_outputs(o, h->stream), "output launch");
}

// Base state: theta_b solves A theta = rhs by iterative refinement.  Each
// pass forms the double-double residual rho of the current theta_b, solves
// A delta = rho by PCG from zero (the per-column right-hand-side mode with the
// intact grid), with the stop relative to ||rho|| rather than to ||rhs||,
// then theta_b += delta; repeated while the residual keeps shrinking.  The
// stop has to follow rho: on a large grid the FP64 residual floor (about
// 1e-11 relative) is reached while the smooth error modes, which the
// residual barely sees, are still well above rounding level; a pass stopped
// at tol ||rhs|| leaves them there.
void base_solve(gpcg_context *h, const double *rhs_host, int max_iter) {
    const int n_bus = h->n_bus;
    DevBuf<double> rhs;
    rhs.upload(rhs_host, n_bus, h->stream);
    DevBuf<int32_t> out1;
    const int32_t minus1 = -1;
    out1.upload(&minus1, 1, h->stream);
    DevBuf<int32_t> it, st;
    it.alloc(1);
    st.alloc(1);
    DevBuf<double> dsum;
    dsum.alloc(2);
    std::vector<double> zero(n_bus, 0.0);
    h->theta_b.upload(zero.data(), n_bus, h->stream);
    DevBuf<double> rho_bus;  // rho in bus numbering (entry 0, the slack, is 0)
    rho_bus.upload(zero.data(), n_bus, h->stream);
    DevSchedule &D = h->schedule_for(1);
    const Work w = context_work(h, 1, 1, D);
    DevBuf<double> xb;  // each pass's correction, by bus
    xb.alloc(n_bus);
    double bnorm2 = 0.0;
    hip_check(gpcg::launch_sumsq(n_bus - 1, rhs.p + 1, dsum.p + 1, h->stream), "sumsq");
    hip_check(hipMemcpyAsync(&bnorm2, dsum.p + 1, sizeof(double), hipMemcpyDeviceToHost, h->stream), "copy");
    hip_check(hipStreamSynchronize(h->stream), "sync");
    double prev = INFINITY;
    h->base_iters = 0;
    for (int pass = 0; pass < 6; ++pass) {
        hip_check(gpcg::launch_base_residual(h->n_r, h->a_rowptr.p, h->a_col.p, h->a_val.p, h->theta_b.p, rhs.p,
                                             nullptr, h->rho_b.p, h->stream),
                  "base residual");
        double rr = 0.0;
        hip_check(gpcg::launch_sumsq(h->n_r, h->rho_b.p, dsum.p, h->stream), "sumsq");
        hip_check(hipMemcpyAsync(&rr, dsum.p, sizeof(double), hipMemcpyDeviceToHost, h->stream), "copy");
        hip_check(hipStreamSynchronize(h->stream), "sync");
        const double rel = bnorm2 > 0.0 ? std::sqrt(rr / bnorm2) : std::sqrt(rr);
        h->base_resid = rel;
        if (!(rel < prev * 0.5) || rel < 1e-16) break;
        prev = rel;
        hip_check(hipMemcpyAsync(rho_bus.p + 1, h->rho_b.p, h->n_r * sizeof(double), hipMemcpyDeviceToDevice,
                                 h->stream),
                  "copy");
        gpcg::PcgParams p = h->params(D, out1.p, 1, rhs.p, 1e-13, max_iter, it.p, st.p);
        p.bus_map = nullptr;  // the correction's right-hand side and result are by internal bus
        p.rhs_cols = rho_bus.p;
        p.rhs_ld = n_bus;
        p.ws = w.ws;
        p.ws_slot = w.ws_slot;
        p.gfac_out = w.gfac;
        p.x_out = xb.p;
        p.add_base = 0;
        hip_check(gpcg::launch_pcg(p, 1, 1, D.ring_max(), false, h->stream), "base pcg");
        hip_check(gpcg::launch_base_accumulate(n_bus, h->theta_b.p, xb.p, h->stream), "base accumulate");
        int its = 0;
        hip_check(hipMemcpyAsync(&its, it.p, sizeof(int), hipMemcpyDeviceToHost, h->stream), "copy");
        hip_check(hipStreamSynchronize(h->stream), "sync");
        h->base_iters += its;
    }
    h->theta_b_host.assign(n_bus, 0.0);
    hip_check(hipMemcpyAsync(h->theta_b_host.data(), h->theta_b.p, n_bus * sizeof(double), hipMemcpyDeviceToHost,
                             h->stream),
              "copy");
    hip_check(hipStreamSynchronize(h->stream), "sync");
}

// ---------------------------------------------------------------------------
// Batches: the scenario lists of several grids solved by one launch of the
// tile kernel, captured once in a HIP graph and replayed.  A batch owns
// everything a replay writes or reads that a later call on one of its
// contexts could reallocate (workspace, scenario order, base residual,
// re-dispatch factors) and holds a reference to the schedules it uses; the
// contexts' matrices and branch tables are read in place, so the contexts
// must outlive the batch.
struct BatchGrid {
    gpcg_context *ctx = nullptr;
    std::shared_ptr<DevSchedule> sched;
    int n_out = 0, tiles = 0;
    const int32_t *outages = nullptr;
    const double *rhs = nullptr;
    double *x_out = nullptr, *flows_out = nullptr, *resid_out = nullptr;
    int32_t *iters_out = nullptr, *status_out = nullptr;
    DevBuf<double> rho_b, gfac;
    DevBuf<int32_t> order, pos;
    // ranking of the scenario queue (rebuilt before every solve from the
    // context's per-outage iteration record)
    DevBuf<uint32_t> keys, keys_sorted;
    DevBuf<int32_t> iota;
    DevBuf<char> temp;
    size_t temp_bytes = 0;
};

struct BatchSpec {
    int n = 0;
    const gpcg_t *ctxs = nullptr;
    const int32_t *n_outs = nullptr;
    const int32_t *const *outages = nullptr;
    const double *const *rhs = nullptr;
    double *const *x_out = nullptr;
    double *const *flows_out = nullptr;
    double *const *resid_out = nullptr;
    int32_t *const *iters_out = nullptr;
    int32_t *const *status_out = nullptr;
};

}  // namespace

struct gpcg_batch {
    int device = 0, S = 1, ring = 1, n_waves = 0, max_iter = 1;
    double tol = 0.0;
    hipStream_t stream = nullptr;
    std::vector<std::unique_ptr<BatchGrid>> g;  // heaviest grid first
    DevBuf<gpcg::PcgParams> params;
    DevBuf<double> ws;                  // the waves' slots, sized for the largest grid
    DevBuf<int32_t> queues;             // one queue counter per grid
    DevBuf<unsigned long long> sweeps;  // iterations summed over the waves
    hipStream_t outer = nullptr;  // the contexts' stream; the batch works on a stream of its own
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~gpcg_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

namespace {

// Build a batch without its graph: per grid the schedules for S, its own
// workspace, the scenario order (once), the kernel parameters.
std::unique_ptr<gpcg_batch> batch_build(const BatchSpec &sp, int S, double tol, int max_iter, int look = 0) {
    if (sp.n < 1) fail(GPCG_E_ARG, "a batch needs at least one context");
    if (S < 1 || S > 64 || (S & (S - 1))) fail(GPCG_E_ARG, "block must be a power of two in [1, 64]");
    if (max_iter < 1) fail(GPCG_E_ARG, "max_iter must be >= 1");
    if (!(tol >= 0.0) || !std::isfinite(tol)) fail(GPCG_E_ARG, "tol must be finite and >= 0");
    auto b = std::make_unique<gpcg_batch>();
    b->S = S;
    b->tol = tol;
    b->max_iter = max_iter;
    for (int i = 0; i < sp.n; ++i) {
        gpcg_context *h = sp.ctxs[i];
        if (!h) fail(GPCG_E_ARG, "context is NULL");
        if (i == 0) {
            b->device = h->device;
            b->outer = h->stream;
        } else if (h->device != b->device || h->stream != b->outer) {
            fail(GPCG_E_ARG, "the contexts of a batch must share a device and a stream");
        }
        const int n_out = sp.n_outs[i];
        if (n_out < 0) fail(GPCG_E_ARG, "n_out < 0");
        if (n_out && (!sp.outages[i] || !sp.rhs[i] || !sp.x_out[i] || !sp.iters_out[i] || !sp.status_out[i]))
            fail(GPCG_E_ARG, "a required pointer is NULL");
        if (sp.flows_out && sp.flows_out[i] && h->kind != GPCG_KIND_BP)
            fail(GPCG_E_ARG, "flows are only defined for a B' context");
        auto G = std::make_unique<BatchGrid>();
        G->ctx = h;
        G->n_out = n_out;
        G->tiles = (n_out + S - 1) / S;
        G->outages = sp.outages[i];
        G->rhs = sp.rhs[i];
        G->x_out = sp.x_out[i];
        G->flows_out = sp.flows_out ? sp.flows_out[i] : nullptr;
        G->resid_out = sp.resid_out ? sp.resid_out[i] : nullptr;
        G->iters_out = sp.iters_out[i];
        G->status_out = sp.status_out[i];
        b->g.push_back(std::move(G));
    }
    hip_check(hipSetDevice(b->device), "hipSetDevice");
    // a stream of the batch's own (a graph cannot be captured on the null
    // stream), default priority, ordered against the contexts' stream
    hip_check(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking), "batch stream");
    hip_check(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming), "batch event");
    hip_check(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming), "batch event");
    hip_check(hipEventRecord(b->ev_in, b->outer), "event");
    hip_check(hipStreamWaitEvent(b->stream, b->ev_in, 0), "stream wait");
    // heaviest first: the tiles of big grids run longest
    std::stable_sort(b->g.begin(), b->g.end(),
                     [](const std::unique_ptr<BatchGrid> &x, const std::unique_ptr<BatchGrid> &y) {
                         return x->ctx->n_r > y->ctx->n_r;
                     });
    // schedules, ring and workspace slot of the largest grid, wave count
    size_t slot = 0;
    long columns = 0;
    for (auto &G : b->g) {
        gpcg_context *h = G->ctx;
        G->sched = h->schedule_ptr(S, look);
        b->ring = std::max(b->ring, G->sched->ring_max());
        slot = std::max(slot, h->ws_slot(S));
        columns += G->tiles;
    }
    const int cap = S == 1 ? 1 : gpcg::pcg_max_waves(S, b->ring);
    if (cap <= 0) fail(GPCG_E_HIP, "occupancy query of the PCG kernel failed");
    b->n_waves = (int)std::max<long>(1, std::min<long>(cap, columns));
    b->ws.alloc((size_t)b->n_waves * slot);
    b->queues.alloc(b->g.size());
    b->sweeps.alloc(1);
    std::vector<gpcg::PcgParams> prm;
    int gi = 0;
    for (auto &G : b->g) {
        gpcg_context *h = G->ctx;
        G->rho_b.alloc(h->n_r);
        G->gfac.alloc(std::max(G->n_out, 1));
        gpcg::PcgParams p = h->params(*G->sched, G->outages, G->n_out, G->rhs, tol, max_iter, G->iters_out,
                                      G->status_out);
        p.ws = b->ws.p;
        p.ws_slot = slot;
        p.queue = b->queues.p + gi++;
        p.sweeps = b->sweeps.p;
        p.rho_b = G->rho_b.p;
        p.gfac_out = G->gfac.p;
        p.x_out = G->x_out;
        p.zero_start = h->zero_start;
        p.add_base = h->zero_start ? 0 : 1;
        if (needs_order(S, G->n_out)) {
            const int n = G->n_out;
            G->keys.alloc(n);
            G->keys_sorted.alloc(n);
            G->iota.alloc(n);
            G->order.alloc(n);
            G->pos.alloc(n);
            G->temp_bytes = gpcg::sort_temp_bytes(n);
            G->temp.alloc(std::max<size_t>(G->temp_bytes, 1));
            p.order = G->order.p;
        }
        prm.push_back(p);
    }
    b->params.upload(prm.data(), prm.size(), b->stream);
    hip_check(hipStreamSynchronize(b->stream), "batch upload");
    return b;
}

// Rank every grid's scenario queue, most expected work first: by the
// iterations each outage took in its context's previous solve (batch or
// single), by the analytic key where there is no record.  Enqueued before
// each solve, outside the captured graph (the sort is a library call).
void batch_order(gpcg_batch *b) {
    for (auto &G : b->g) {
        if (!G->order.p) continue;
        gpcg_context *h = G->ctx;
        hip_check(gpcg::launch_order(G->n_out, G->outages, h->m, h->br_from.p, h->br_to.p, h->br_b.p, h->isl_lo.p,
                                     h->isl_hi.p, h->theta_b.p, h->hist_base.p, G->keys.p, G->keys_sorted.p,
                                     G->iota.p, G->order.p, G->pos.p, G->temp.p, G->temp_bytes, b->stream),
                  "scenario ordering");
    }
}

// Everything one solve of the batch enqueues (what the graph captures):
// kernels only, no memory set or copy nodes.
void batch_enqueue(gpcg_batch *b) {
    for (auto &G : b->g) {
        gpcg_context *h = G->ctx;
        if (G->n_out == 0 || h->zero_start) continue;
        hip_check(gpcg::launch_base_residual(h->n_r, h->a_rowptr.p, h->a_col.p, h->a_val.p, h->theta_b.p, G->rhs,
                                             h->bus_map.p, G->rho_b.p, b->stream),
                  "base residual");
    }
    // streamed vectors once every ranked grid has an iteration record (the
    // captured solve, after the eager one), as for a single context
    bool ranked = false, recorded = true;
    for (auto &G : b->g)
        if (G->order.p) {
            ranked = true;
            recorded = recorded && G->ctx->rec_base;
        }
    hip_check(gpcg::launch_pcg_multi(b->params.p, (int)b->g.size(), b->S, b->n_waves, b->ring,
                                     ranked && recorded && streams_vectors(b->ws.n), b->stream),
              "batch launch");
    for (auto &G : b->g) {
        if (!G->order.p) continue;
        hip_check(gpcg::launch_record_iters(G->n_out, G->outages, G->ctx->m, G->iters_out, G->ctx->hist_base.p,
                                            b->stream),
                  "iteration records");
        G->ctx->rec_base = true;
    }
    for (auto &G : b->g) {
        gpcg_context *h = G->ctx;
        if (G->n_out == 0) continue;
        gpcg::OutParams o{};
        o.n_r = h->n_r;
        o.n_bus = h->n_bus;
        o.m = h->m;
        o.kind = h->kind;
        o.n_out = G->n_out;
        o.bus_map = h->bus_map.p;
        o.cbr_from = h->cbr_from.p;
        o.cbr_to = h->cbr_to.p;
        o.a_rowptr = h->a_rowptr.p;
        o.a_col = h->a_col.p;
        o.a_val = h->a_val.p;
        o.br_from = h->br_from.p;
        o.br_to = h->br_to.p;
        o.br_x = h->br_x.p;
        o.br_b = h->br_b.p;
        o.pre_bus = h->pre_bus.p;
        o.isl_lo = h->isl_lo.p;
        o.isl_hi = h->isl_hi.p;
        o.theta_b = h->theta_b.p;
        o.rhs = G->rhs;
        o.add_base = h->zero_start ? 0 : 1;
        o.outages = G->outages;
        o.status = G->status_out;
        o.gfac = G->gfac.p;
        o.x_out = G->x_out;
        o.flows_out = G->flows_out;
        o.resid_out = G->resid_out;
        o.island_out = nullptr;
        hip_check(gpcg::launch_outputs(o, b->stream), "batch outputs");
    }
}

}  // namespace

// ===========================================================================
extern "C" {

const char *gpcg_last_error(void) { return g_last_error.c_str(); }

int gpcg_assemble(int32_t n_bus, int32_t m, const int32_t *from, const int32_t *to, const double *x,
                  const double *shunt, const int32_t *perm, int32_t *rowptr, int32_t *col, double *val, int32_t cap,
                  int32_t *nnz_out) {
    return guarded([&] {
        if (!x || !rowptr || !col || !val || !nnz_out) fail(GPCG_E_ARG, "NULL argument");
        check_branches(n_bus, m, from, to, x);
        std::vector<int32_t> rp, c, f2, t2;
        std::vector<double> v, sh2;
        const int32_t *ff = from, *tt = to;
        const double *sh = shunt;
        if (perm) {  // rows in perm's order: relabel the buses by their row
            const std::vector<int32_t> inv = invert_perm(n_bus, perm);
            f2.resize(m);
            t2.resize(m);
            for (int e = 0; e < m; ++e) {
                f2[e] = inv[from[e]];
                t2[e] = inv[to[e]];
            }
            ff = f2.data();
            tt = t2.data();
            if (shunt) {
                sh2.assign(n_bus, 0.0);
                for (int k = 0; k < n_bus; ++k) sh2[inv[k]] = shunt[k];
                sh = sh2.data();
            }
        }
        const int nnz = assemble(n_bus, m, ff, tt, x, sh, rp, c, v);
        if (nnz > cap) fail(GPCG_E_ARG, "output capacity too small");
        std::copy(rp.begin(), rp.end(), rowptr);
        std::copy(c.begin(), c.end(), col);
        std::copy(v.begin(), v.end(), val);
        *nnz_out = nnz;
    });
}

int gpcg_rcm(int32_t n_bus, int32_t m, const int32_t *from, const int32_t *to, int32_t *perm) {
    return guarded([&] {
        if (!perm) fail(GPCG_E_ARG, "perm is NULL");
        check_branches(n_bus, m, from, to, nullptr);
        const std::vector<int32_t> p = rcm_order(n_bus, m, from, to);
        std::copy(p.begin(), p.end(), perm);
    });
}

int gpcg_ilu0(const gpcg_csr *A, int32_t *l_rowptr, int32_t *l_col, double *l_val, int32_t *nnz_l,
              int32_t *u_rowptr, int32_t *u_col, double *u_val, int32_t *nnz_u) {
    return guarded([&] {
        if (!A || !l_rowptr || !l_col || !l_val || !nnz_l || !u_rowptr || !u_col || !u_val || !nnz_u)
            fail(GPCG_E_ARG, "NULL argument");
        check_csr(A, "A", A->n);
        std::vector<double> F;
        std::vector<int> dp;
        ilu0(*A, F, dp);
        int nl = 0, nu = 0;
        l_rowptr[0] = u_rowptr[0] = 0;
        for (int i = 0; i < A->n; ++i) {
            for (int e = A->rowptr[i]; e < A->rowptr[i + 1]; ++e) {
                if (A->col[e] < i) {
                    l_col[nl] = A->col[e];
                    l_val[nl++] = F[e];
                } else {
                    u_col[nu] = A->col[e];
                    u_val[nu++] = F[e];
                }
            }
            l_rowptr[i + 1] = nl;
            u_rowptr[i + 1] = nu;
        }
        *nnz_l = nl;
        *nnz_u = nu;
    });
}

int gpcg_topology(int32_t n_bus, int32_t m, const int32_t *from, const int32_t *to, uint8_t *is_bridge,
                  int32_t *pre, int32_t *subtree, int32_t *island_lo, int32_t *island_hi) {
    return guarded([&] {
        check_branches(n_bus, m, from, to, nullptr);
        Topology T = topology(n_bus, m, from, to);
        if (is_bridge) std::copy(T.is_bridge.begin(), T.is_bridge.end(), is_bridge);
        if (pre) std::copy(T.pre.begin(), T.pre.end(), pre);
        if (subtree) std::copy(T.sub.begin(), T.sub.end(), subtree);
        if (island_lo) std::copy(T.lo.begin(), T.lo.end(), island_lo);
        if (island_hi) std::copy(T.hi.begin(), T.hi.end(), island_hi);
    });
}

int gpcg_setup(gpcg_t *out, int32_t n_bus, int32_t m, const int32_t *br_from, const int32_t *br_to,
               const double *br_x, const gpcg_csr *A, const gpcg_csr *L, const gpcg_csr *U, const double *base_rhs,
               const double *theta_base, const gpcg_options *opt, void *stream) {
    if (out) *out = nullptr;
    return guarded([&] {
        if (!out) fail(GPCG_E_ARG, "out is NULL");
        if (n_bus < 2) fail(GPCG_E_ARG, "need at least two buses");
        if (n_bus >= gpcg::kBwdRowMask) fail(GPCG_E_UNSUPPORTED, "at most 2^20 - 2 buses");
        if (!br_x) fail(GPCG_E_ARG, "br_x is NULL");
        check_branches(n_bus, m, br_from, br_to, br_x);
        const int nr = n_bus - 1;
        check_csr(A, "A", nr);
        if (!theta_base && !base_rhs) fail(GPCG_E_ARG, "either base_rhs or theta_base is required");
        gpcg_options o{};
        if (opt) o = *opt;
        if (o.kind != GPCG_KIND_BP && o.kind != GPCG_KIND_BPP) fail(GPCG_E_ARG, "unknown kind");
        const int S = o.block ? o.block : 64;
        if (S < 1 || S > 64 || (S & (S - 1))) fail(GPCG_E_ARG, "block must be a power of two in [1, 64]");
        if ((L == nullptr) != (U == nullptr)) fail(GPCG_E_ARG, "give both factors L and U, or neither");
        if (o.reorder && o.perm) fail(GPCG_E_ARG, "give perm or ask for reorder, not both");
        if (o.reorder && L) fail(GPCG_E_ARG, "reorder forms its own factors: L and U must be NULL");
        // The row order: the caller's perm, the library's reverse Cuthill-McKee
        // order (reorder; A is then given in bus order and permuted here), or
        // the bus order.  inv turns a caller's bus into its internal bus.
        std::vector<int32_t> perm, inv;
        if (o.perm) {
            perm.assign(o.perm, o.perm + nr);
            inv = invert_perm(n_bus, o.perm);
        } else if (o.reorder) {
            perm = rcm_order(n_bus, m, br_from, br_to);
            inv = invert_perm(n_bus, perm.data());
        }
        CsrH Ah, Lh, Uh;
        if (o.reorder) {
            std::vector<std::vector<std::pair<int, double>>> rows(nr);
            for (int i = 0; i < nr; ++i)
                for (int e = A->rowptr[i]; e < A->rowptr[i + 1]; ++e)
                    rows[inv[i + 1] - 1].push_back({inv[A->col[e] + 1] - 1, A->val[e]});
            Ah.rowptr.assign(nr + 1, 0);
            for (int i = 0; i < nr; ++i) {
                std::sort(rows[i].begin(), rows[i].end());
                for (auto &cv : rows[i]) {
                    Ah.col.push_back(cv.first);
                    Ah.val.push_back(cv.second);
                }
                Ah.rowptr[i + 1] = (int32_t)Ah.col.size();
            }
        } else {
            Ah.rowptr.assign(A->rowptr, A->rowptr + nr + 1);
            Ah.col.assign(A->col, A->col + A->nnz);
            Ah.val.assign(A->val, A->val + A->nnz);
        }
        gpcg_csr Av{nr, (int32_t)Ah.col.size(), Ah.rowptr.data(), Ah.col.data(), Ah.val.data()};
        A = &Av;
        if (!L) {  // the base-case ILU(0) of A in row order (Section IV.B)
            std::vector<double> F;
            std::vector<int> dp;
            ilu0(Av, F, dp);
            Lh.rowptr.assign(nr + 1, 0);
            Uh.rowptr.assign(nr + 1, 0);
            for (int i = 0; i < nr; ++i) {
                for (int e = Ah.rowptr[i]; e < Ah.rowptr[i + 1]; ++e) {
                    CsrH &T = Ah.col[e] < i ? Lh : Uh;
                    T.col.push_back(Ah.col[e]);
                    T.val.push_back(F[e]);
                }
                Lh.rowptr[i + 1] = (int32_t)Lh.col.size();
                Uh.rowptr[i + 1] = (int32_t)Uh.col.size();
            }
        } else {
            check_csr(L, "L", nr);
            check_csr(U, "U", nr);
            Lh.rowptr.assign(L->rowptr, L->rowptr + nr + 1);
            Lh.col.assign(L->col, L->col + L->nnz);
            Lh.val.assign(L->val, L->val + L->nnz);
            Uh.rowptr.assign(U->rowptr, U->rowptr + nr + 1);
            Uh.col.assign(U->col, U->col + U->nnz);
            Uh.val.assign(U->val, U->val + U->nnz);
        }
        gpcg_csr Lv{nr, (int32_t)Lh.col.size(), Lh.rowptr.data(), Lh.col.data(), Lh.val.data()};
        gpcg_csr Uv{nr, (int32_t)Uh.col.size(), Uh.rowptr.data(), Uh.col.data(), Uh.val.data()};
        L = &Lv;
        U = &Uv;
        // branch endpoints as internal buses (the caller's when no perm)
        std::vector<int32_t> ifrom(br_from, br_from + m), ito(br_to, br_to + m);
        if (!inv.empty())
            for (int e = 0; e < m; ++e) {
                ifrom[e] = inv[br_from[e]];
                ito[e] = inv[br_to[e]];
            }
        // factor shapes: L strictly lower, U upper with a positive diagonal first
        std::vector<double> invdiag(nr);
        std::vector<int32_t> us_rowptr(nr + 1, 0), us_col;
        std::vector<double> us_val;
        for (int i = 0; i < nr; ++i) {
            for (int e = L->rowptr[i]; e < L->rowptr[i + 1]; ++e)
                if (L->col[e] >= i) fail(GPCG_E_PATTERN, "L must be strictly lower triangular");
            if (U->rowptr[i + 1] == U->rowptr[i] || U->col[U->rowptr[i]] != i)
                fail(GPCG_E_PATTERN, "U must hold the diagonal as the first entry of each row");
            const double d = U->val[U->rowptr[i]];
            if (!(d > 0.0)) fail(GPCG_E_PIVOT, "U has a zero or negative pivot at row " + std::to_string(i));
            invdiag[i] = 1.0 / d;
            for (int e = U->rowptr[i] + 1; e < U->rowptr[i + 1]; ++e) {
                us_col.push_back(U->col[e]);
                us_val.push_back(U->val[e]);
            }
            us_rowptr[i + 1] = (int32_t)us_col.size();
        }
        bool has_diag = true;
        int bw = 0;
        for (int i = 0; i < nr; ++i) {
            bool d = false;
            for (int e = A->rowptr[i]; e < A->rowptr[i + 1]; ++e) {
                d |= A->col[e] == i;
                bw = std::max(bw, std::abs(A->col[e] - i));
            }
            has_diag &= d;
        }
        if (!has_diag) fail(GPCG_E_PATTERN, "A lacks a diagonal entry");

        auto h = std::make_unique<gpcg_context>();
        hip_check(hipGetDevice(&h->device), "hipGetDevice");
        {  // the fixed scratch's address on this device (looked up once per device)
            void *fixed = nullptr;
            hip_check(gpcg::static_scratch(&fixed), "static scratch");
        }
        h->stream = (hipStream_t)stream;
        h->n_bus = n_bus;
        h->m = m;
        h->n_r = nr;
        h->kind = o.kind;
        h->S = S;
        h->look = o.lookahead > 0 ? o.lookahead : 256;
        h->zero_start = o.zero_start ? 1 : 0;
        h->bandwidth = bw;
        h->nnz_a = A->nnz;
        h->nnz_l = L->nnz;
        h->nnz_u = U->nnz;
        h->perm = perm;
        h->inv = inv;
        h->topo = topology(n_bus, m, ifrom.data(), ito.data());
        // dependency lists for the schedules (backward on mirrored indices)
        h->deps_f.assign(nr, {});
        h->deps_b.assign(nr, {});
        for (int i = 0; i < nr; ++i) {
            for (int e = L->rowptr[i]; e < L->rowptr[i + 1]; ++e) h->deps_f[i].push_back(L->col[e]);
            for (int e = us_rowptr[i]; e < us_rowptr[i + 1]; ++e) h->deps_b[nr - 1 - i].push_back(nr - 1 - us_col[e]);
        }
        h->hA.rowptr.assign(A->rowptr, A->rowptr + nr + 1);
        h->hA.col.assign(A->col, A->col + A->nnz);
        h->hA.val.assign(A->val, A->val + A->nnz);
        h->hL.rowptr.assign(L->rowptr, L->rowptr + nr + 1);
        h->hL.col.assign(L->col, L->col + L->nnz);
        h->hL.val.assign(L->val, L->val + L->nnz);
        h->hU.rowptr = us_rowptr;
        h->hU.col = us_col;
        h->hU.val = us_val;
        h->h_invdiag = invdiag;
        h->sym_factors = factors_symmetric(h->hL, h->hU, invdiag);
        h->h_prerow.resize(nr);
        for (int i = 0; i < nr; ++i) h->h_prerow[i] = h->topo.pre[i + 1];
        hipStream_t st = h->stream;
        h->a_rowptr.upload(A->rowptr, nr + 1, st);
        h->a_col.upload(A->col, A->nnz, st);
        h->a_val.upload(A->val, A->nnz, st);
        h->l_rowptr.upload(L->rowptr, nr + 1, st);
        h->l_col.upload(L->col, L->nnz, st);
        h->l_val.upload(L->val, L->nnz, st);
        h->u_rowptr.upload(us_rowptr.data(), nr + 1, st);
        h->u_col.upload(us_col.data(), us_col.size(), st);
        h->u_val.upload(us_val.data(), us_val.size(), st);
        h->u_invdiag.upload(invdiag.data(), nr, st);
        std::vector<double> b(m);
        for (int e = 0; e < m; ++e) b[e] = 1.0 / br_x[e];
        h->br_from.upload(ifrom.data(), m, st);
        h->br_to.upload(ito.data(), m, st);
        h->cbr_from.upload(br_from, m, st);
        h->cbr_to.upload(br_to, m, st);
        h->br_x.upload(br_x, m, st);
        h->br_b.upload(b.data(), m, st);
        std::vector<int32_t> prerow(nr);
        for (int i = 0; i < nr; ++i) prerow[i] = h->topo.pre[i + 1];
        h->pre_row.upload(prerow.data(), nr, st);
        h->pre_bus.upload(h->topo.pre.data(), n_bus, st);
        {  // pre-order numbers by the caller's bus, and internal bus -> caller's bus
            std::vector<int32_t> cpre(n_bus);
            for (int k = 0; k < n_bus; ++k) cpre[k] = h->topo.pre[inv.empty() ? k : inv[k]];
            h->cpre_bus.upload(cpre.data(), n_bus, st);
            if (!perm.empty()) {
                std::vector<int32_t> map(n_bus, 0);
                for (int k = 0; k < nr; ++k) map[k + 1] = perm[k];
                h->bus_map.upload(map.data(), n_bus, st);
            }
        }
        h->isl_lo.upload(h->topo.lo.data(), m, st);
        h->isl_hi.upload(h->topo.hi.data(), m, st);
        {  // branches incident to each bus, for gathers over a bus's branches
            std::vector<int32_t> ptr(n_bus + 1, 0), br(2 * (size_t)m);
            for (int e = 0; e < m; ++e) {
                ++ptr[br_from[e] + 1];
                ++ptr[br_to[e] + 1];
            }
            for (int k = 0; k < n_bus; ++k) ptr[k + 1] += ptr[k];
            std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
            for (int e = 0; e < m; ++e) {
                br[fill[br_from[e]]++] = e;
                br[fill[br_to[e]]++] = e;
            }
            h->inc_ptr.upload(ptr.data(), ptr.size(), st);
            h->inc_br.upload(br.data(), br.size(), st);
        }
        h->rho_b.alloc(nr);
        h->queue.alloc(1);
        h->sweeps.alloc(1);
        {  // no iteration records yet
            const std::vector<int32_t> none(m + 1, -1);
            h->hist_base.upload(none.data(), m + 1, st);
            h->hist_cols.upload(none.data(), m + 1, st);
        }
        hip_check(hipStreamSynchronize(st), "setup upload");
        h->schedule_for(S);
        if (theta_base) {
            std::vector<double> t(n_bus, 0.0);  // by internal bus
            for (int k = 1; k < n_bus; ++k) t[h->internal_bus(k)] = theta_base[k];
            h->theta_b.upload(t.data(), n_bus, st);
            h->theta_b_host = t;
            hip_check(hipStreamSynchronize(st), "theta upload");
        } else {
            std::vector<double> r(n_bus, 0.0);
            for (int k = 0; k < n_bus; ++k) r[h->internal_bus(k)] = base_rhs[k];
            base_solve(h.get(), r.data(), o.base_max_iter > 0 ? o.base_max_iter : 20000);
        }
        *out = h.release();
    });
}

void gpcg_destroy(gpcg_t h) {
    if (!h) return;
    try {
        (void)hipSetDevice(h->device);
        (void)hipStreamSynchronize(h->stream);
        delete h;
    } catch (...) {
    }
}

int gpcg_get_info(gpcg_t h, gpcg_info *info) {
    return guarded([&] {
        if (!h || !info) fail(GPCG_E_ARG, "NULL argument");
        DevSchedule &D = h->schedule_for(h->S);
        gpcg_info I{};
        I.n_bus = h->n_bus;
        I.m = h->m;
        I.n_r = h->n_r;
        I.nnz_a = h->nnz_a;
        I.nnz_l = h->nnz_l;
        I.nnz_u = h->nnz_u;
        I.bandwidth = h->bandwidth;
        I.block = h->S;
        I.rows_per_step = D.R;
        I.ring_fwd = D.f.ring;
        I.ring_bwd = D.b.ring;
        I.steps_fwd = D.f.steps;
        I.steps_bwd = D.b.steps;
        I.n_bridges = h->topo.n_bridges;
        I.base_iters = h->base_iters;
        I.base_resid = h->base_resid;
        I.sym_factors = h->sym_factors ? 1 : 0;
        *info = I;
    });
}

int gpcg_get_base(gpcg_t h, uint8_t *is_bridge, double *theta_base) {
    return guarded([&] {
        if (!h) fail(GPCG_E_ARG, "NULL context");
        if (is_bridge) std::copy(h->topo.is_bridge.begin(), h->topo.is_bridge.end(), is_bridge);
        if (theta_base)
            for (int k = 0; k < h->n_bus; ++k) theta_base[k] = h->theta_b_host[h->internal_bus(k)];
    });
}

int gpcg_bridge_flags(gpcg_t h, uint8_t *is_bridge) {
    return guarded([&] {
        if (!h || !is_bridge) fail(GPCG_E_ARG, "NULL argument");
        std::copy(h->topo.is_bridge.begin(), h->topo.is_bridge.end(), is_bridge);
    });
}

int gpcg_get_perm(gpcg_t h, int32_t *perm) {
    return guarded([&] {
        if (!h || !perm) fail(GPCG_E_ARG, "NULL argument");
        for (int k = 0; k < h->n_r; ++k) perm[k] = h->perm.empty() ? k + 1 : h->perm[k];
    });
}

int gpcg_solve_contingencies(gpcg_t h, int32_t n_out, const int32_t *outages, const double *rhs, double tol,
                             int32_t max_iter, double *x_out, double *flows_out, int32_t *iters_out,
                             int32_t *status_out, uint8_t *island_out, double *resid_out) {
    return guarded([&] {
        if (!h) fail(GPCG_E_ARG, "context is NULL");
        run_solve(h, h->S, n_out, outages, rhs, tol, max_iter, x_out, flows_out, iters_out, status_out, island_out,
                  resid_out);
    });
}

int gpcg_solve_contingencies_noalloc(gpcg_t h, int32_t n_out, const int32_t *outages, const double *rhs, double tol,
                                     int32_t max_iter, double *x_out, double *flows_out, int32_t *iters_out,
                                     int32_t *status_out, uint8_t *island_out, double *resid_out) {
    return guarded([&] {
        if (!h) fail(GPCG_E_ARG, "context is NULL");
        run_solve(h, h->S, n_out, outages, rhs, tol, max_iter, x_out, flows_out, iters_out, status_out, island_out,
                  resid_out, nullptr, 0, true);
    });
}

int gpcg_solve_rhs(gpcg_t h, int32_t n_out, const int32_t *outages, const double *rhs_cols, int32_t ld, double tol,
                   int32_t max_iter, double *x_out, int32_t *iters_out, int32_t *status_out, uint8_t *island_out,
                   double *resid_out) {
    return guarded([&] {
        if (!h) fail(GPCG_E_ARG, "context is NULL");
        if (!rhs_cols) fail(GPCG_E_ARG, "rhs_cols is NULL");
        run_solve(h, h->S, n_out, outages, nullptr, tol, max_iter, x_out, nullptr, iters_out, status_out, island_out,
                  resid_out, rhs_cols, ld);
    });
}

int gpcg_overload_gradients(gpcg_t h, int32_t n_out, const int32_t *outages, const double *rhs,
                            const double *flow_limit, double kappa, double tol, int32_t max_iter, double *loss_out,
                            double *grad_p_out, double *grad_x_out, int32_t *iters_out, int32_t *status_out) {
    return guarded([&] {
        if (!h) fail(GPCG_E_ARG, "context is NULL");
        if (h->kind != GPCG_KIND_BP) fail(GPCG_E_ARG, "the overload loss is defined on a B' context");
        if (n_out < 0) fail(GPCG_E_ARG, "n_out < 0");
        if (!outages || !rhs || !flow_limit || !loss_out || !iters_out || !status_out)
            fail(GPCG_E_ARG, "a required pointer is NULL");
        if (!(kappa > 0.0) || !std::isfinite(kappa)) fail(GPCG_E_ARG, "kappa must be finite and > 0");
        if (n_out == 0) return;
        hip_check(hipSetDevice(h->device), "hipSetDevice");
        const size_t nb = (size_t)n_out * h->n_bus, nm = (size_t)n_out * h->m;
        if (h->ov_theta.n < nb) {
            h->ov_theta.alloc(nb);
            h->ov_g.alloc(nb);
            h->ov_lambda.alloc(nb);
        }
        if (h->ov_flows.n < nm) h->ov_flows.alloc(nm);
        // forward: the scenario angles and flows (recomputed, nothing stored
        // from an earlier call)
        run_solve(h, h->S, n_out, outages, rhs, tol, max_iter, h->ov_theta.p, h->ov_flows.p, iters_out, status_out,
                  nullptr, nullptr);
        gpcg::OverloadParams o{};
        o.n_bus = h->n_bus;
        o.m = h->m;
        o.n_out = n_out;
        o.kappa = kappa;
        o.br_from = h->cbr_from.p;  // every array of this call is by the caller's bus
        o.br_to = h->cbr_to.p;
        o.br_x = h->br_x.p;
        o.inc_ptr = h->inc_ptr.p;
        o.inc_br = h->inc_br.p;
        o.pre_bus = h->cpre_bus.p;
        o.isl_lo = h->isl_lo.p;
        o.isl_hi = h->isl_hi.p;
        o.outages = outages;
        o.P = rhs;
        o.F = flow_limit;
        o.theta = h->ov_theta.p;
        o.flows = h->ov_flows.p;
        o.lambda = h->ov_lambda.p;
        o.g = h->ov_g.p;
        o.loss = loss_out;
        o.grad_p = grad_p_out;
        o.grad_x = grad_x_out;
        hip_check(gpcg::launch_overload_seed(o, h->stream), "overload seed");
        if (!grad_p_out && !grad_x_out) return;
        // adjoint: A_c[M,M] lambda = g_M with the same preconditioner
        run_solve(h, h->S, n_out, outages, nullptr, tol, max_iter, h->ov_lambda.p, nullptr, iters_out + n_out,
                  status_out + n_out, nullptr, nullptr, h->ov_g.p, h->n_bus);
        hip_check(gpcg::launch_overload_grads(o, h->stream), "overload gradients");
    });
}

int gpcg_weighted_rows(gpcg_t h, int32_t n_rows, int32_t n_cols, const double *a, int32_t lda, const double *w,
                       double *out) {
    return guarded([&] {
        if (!h) fail(GPCG_E_ARG, "context is NULL");
        if (n_rows < 0 || n_cols < 0 || lda < n_cols) fail(GPCG_E_ARG, "bad sizes");
        if ((n_rows && n_cols && (!a || !w)) || (n_cols && !out)) fail(GPCG_E_ARG, "a required pointer is NULL");
        hip_check(hipSetDevice(h->device), "hipSetDevice");
        hip_check(gpcg::launch_weighted_rows(n_rows, n_cols, a, lda, w, out, h->stream), "weighted rows");
    });
}

int gpcg_fdpf(gpcg_t bp, gpcg_t bpp, int32_t n_out, const int32_t *outages, const double *P, const double *Q,
              const double *theta0, const double *V0, int32_t n_outer, double tol, int32_t max_iter,
              double *theta_out, double *V_out, int32_t *iters_out, int32_t *status_out) {
    return guarded([&] {
        if (!bp || !bpp) fail(GPCG_E_ARG, "context is NULL");
        if (bp->kind != GPCG_KIND_BP || bpp->kind != GPCG_KIND_BPP)
            fail(GPCG_E_ARG, "the first context must be B' and the second B''");
        if (bp->n_bus != bpp->n_bus || bp->m != bpp->m) fail(GPCG_E_ARG, "the two contexts hold different grids");
        if (bp->stream != bpp->stream || bp->device != bpp->device)
            fail(GPCG_E_ARG, "the two contexts must share a device and a stream");
        if (n_out < 0 || n_outer < 1) fail(GPCG_E_ARG, "n_out < 0 or n_outer < 1");
        if (n_out == 0) return;
        if (!outages || !P || !Q || !theta0 || !V0 || !theta_out || !V_out || !iters_out || !status_out)
            fail(GPCG_E_ARG, "a required pointer is NULL");
        hip_check(hipSetDevice(bp->device), "hipSetDevice");
        if (!bpp->diag_bus.p) {
            std::vector<double> d(bpp->n_bus, 0.0);
            for (int i = 0; i < bpp->n_r; ++i)
                for (int e = bpp->hA.rowptr[i]; e < bpp->hA.rowptr[i + 1]; ++e)
                    if (bpp->hA.col[e] == i) d[bpp->perm.empty() ? i + 1 : bpp->perm[i]] = bpp->hA.val[e];
            bpp->diag_bus.upload(d.data(), d.size(), bpp->stream);
            hip_check(hipStreamSynchronize(bpp->stream), "diagonal upload");
        }
        const size_t nb = (size_t)n_out * bp->n_bus;
        if (bp->fd_rhs.n < nb) {
            bp->fd_rhs.alloc(nb);
            bp->fd_dx.alloc(nb);
        }
        if (bp->fd_gfac.n < (size_t)n_out) {
            bp->fd_gfac.alloc(n_out);
            bp->fd_nogen.alloc(n_out);
            bp->fd_it.alloc(n_out);
            bp->fd_st.alloc(n_out);
        }
        gpcg::FdpfParams f{};
        f.n_bus = bp->n_bus;
        f.m = bp->m;
        f.n_out = n_out;
        f.br_from = bp->cbr_from.p;  // every array of this call is by the caller's bus
        f.br_to = bp->cbr_to.p;
        f.br_b = bp->br_b.p;
        f.inc_ptr = bp->inc_ptr.p;
        f.inc_br = bp->inc_br.p;
        f.pre_bus = bp->cpre_bus.p;
        f.isl_lo = bp->isl_lo.p;
        f.isl_hi = bp->isl_hi.p;
        f.outages = outages;
        f.P = P;
        f.Q = Q;
        f.diag_bpp = bpp->diag_bus.p;
        f.theta0 = theta0;
        f.V0 = V0;
        f.theta = theta_out;
        f.V = V_out;
        f.rhs = bp->fd_rhs.p;
        f.dx = bp->fd_dx.p;
        f.gfac = bp->fd_gfac.p;
        f.nogen = bp->fd_nogen.p;
        f.iters = iters_out;
        f.status = status_out;
        f.it_step = bp->fd_it.p;
        f.st_step = bp->fd_st.p;
        hipStream_t st = bp->stream;
        hip_check(gpcg::launch_fdpf(f, 0, 0, st), "fdpf start");
        for (int k = 0; k < n_outer; ++k) {
            for (int half = 0; half < 2; ++half) {
                gpcg_context *h = half ? bpp : bp;
                hip_check(gpcg::launch_fdpf(f, 1, half, st), "fdpf mismatch");
                run_solve(h, h->S, n_out, outages, nullptr, tol, max_iter, bp->fd_dx.p, nullptr, bp->fd_it.p,
                          bp->fd_st.p, nullptr, nullptr, bp->fd_rhs.p, bp->n_bus);
                hip_check(gpcg::launch_fdpf(f, 2, half, st), "fdpf update");
            }
        }
        hip_check(gpcg::launch_fdpf(f, 3, 0, st), "fdpf finish");
    });
}

int gpcg_screen_overloads(gpcg_t h, int32_t n_out, const double *flows, const double *flow_limit,
                          int32_t *count_out, double *worst_out, int32_t *worst_branch_out) {
    return guarded([&] {
        if (!h) fail(GPCG_E_ARG, "context is NULL");
        if (n_out < 0) fail(GPCG_E_ARG, "n_out < 0");
        if (n_out == 0) return;
        if (!flows || !flow_limit || !count_out || !worst_out || !worst_branch_out)
            fail(GPCG_E_ARG, "a required pointer is NULL");
        hip_check(hipSetDevice(h->device), "hipSetDevice");
        hip_check(gpcg::launch_screen(n_out, h->m, flows, flow_limit, count_out, worst_out, worst_branch_out,
                                      h->stream),
                  "screening");
    });
}

int gpcg_batch_create(gpcg_batch_t *out, int32_t n_ctx, const gpcg_t *ctxs, int32_t block, int32_t lookahead,
                      const int32_t *n_outs,
                      const int32_t *const *outages, const double *const *rhs, double tol, int32_t max_iter,
                      double *const *x_out, double *const *flows_out, int32_t *const *iters_out,
                      int32_t *const *status_out, double *const *resid_out) {
    if (out) *out = nullptr;
    return guarded([&] {
        if (!out || !ctxs || !n_outs || !outages || !rhs || !x_out || !iters_out || !status_out)
            fail(GPCG_E_ARG, "a required pointer is NULL");
        BatchSpec sp;
        sp.n = n_ctx;
        sp.ctxs = ctxs;
        sp.n_outs = n_outs;
        sp.outages = outages;
        sp.rhs = rhs;
        sp.x_out = x_out;
        sp.flows_out = flows_out;
        sp.resid_out = resid_out;
        sp.iters_out = iters_out;
        sp.status_out = status_out;
        if (lookahead < 0) fail(GPCG_E_ARG, "lookahead must be >= 0");
        auto b = batch_build(sp, block, tol, max_iter, lookahead);
        // one eager solve (results valid at once), then the same work captured
        batch_order(b.get());
        batch_enqueue(b.get());
        hip_check(hipStreamSynchronize(b->stream), "batch first solve");
        hip_check(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture");
        try {
            batch_enqueue(b.get());
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(b->stream, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        hip_check(hipStreamEndCapture(b->stream, &b->graph), "end capture");
        hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "graph instantiate");
        hip_check(hipEventRecord(b->ev_out, b->stream), "event");
        hip_check(hipStreamWaitEvent(b->outer, b->ev_out, 0), "stream wait");
        *out = b.release();
    });
}

int gpcg_batch_run(gpcg_batch_t b) {
    return guarded([&] {
        if (!b) fail(GPCG_E_ARG, "batch is NULL");
        hip_check(hipSetDevice(b->device), "hipSetDevice");
        hip_check(hipEventRecord(b->ev_in, b->outer), "event");
        hip_check(hipStreamWaitEvent(b->stream, b->ev_in, 0), "stream wait");
        batch_order(b);
        hip_check(hipGraphLaunch(b->exec, b->stream), "graph launch");
        hip_check(hipEventRecord(b->ev_out, b->stream), "event");
        hip_check(hipStreamWaitEvent(b->outer, b->ev_out, 0), "stream wait");
    });
}

void gpcg_batch_destroy(gpcg_batch_t b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    delete b;
}

int gpcg_batch_tune(int32_t n_ctx, const gpcg_t *ctxs, const int32_t *n_outs, const int32_t *const *outages,
                    const double *const *rhs, double tol, int32_t max_iter, int32_t n_cand, const int32_t *cand,
                    const int32_t *cand_look, int32_t reps, double *ms_out) {
    return guarded([&] {
        if (!ctxs || !n_outs || !outages || !rhs || !cand || !ms_out) fail(GPCG_E_ARG, "a required pointer is NULL");
        if (n_ctx < 1 || n_cand < 1 || reps < 1) fail(GPCG_E_ARG, "need contexts, candidates and reps >= 1");
        // scratch outputs shared by the candidates
        std::vector<DevBuf<double>> xs(n_ctx);
        std::vector<DevBuf<int32_t>> its(n_ctx), sts(n_ctx);
        std::vector<double *> xp(n_ctx);
        std::vector<int32_t *> ip(n_ctx), spp(n_ctx);
        for (int i = 0; i < n_ctx; ++i) {
            if (!ctxs[i]) fail(GPCG_E_ARG, "context is NULL");
            const size_t n = std::max(1, n_outs[i]);
            xs[i].alloc(n * ctxs[i]->n_bus);
            its[i].alloc(n);
            sts[i].alloc(n);
            xp[i] = xs[i].p;
            ip[i] = its[i].p;
            spp[i] = sts[i].p;
        }
        BatchSpec sp;
        sp.n = n_ctx;
        sp.ctxs = ctxs;
        sp.n_outs = n_outs;
        sp.outages = outages;
        sp.rhs = rhs;
        sp.x_out = xp.data();
        sp.iters_out = ip.data();
        sp.status_out = spp.data();
        for (int k = 0; k < n_cand; ++k) {
            const int look_k = cand_look ? cand_look[k] : 0;
            if (look_k < 0) fail(GPCG_E_ARG, "lookahead must be >= 0");
            auto b = batch_build(sp, cand[k], tol, max_iter, look_k);
            batch_order(b.get());
            batch_enqueue(b.get());  // warm-up
            hipEvent_t e0, e1;
            hip_check(hipEventCreate(&e0), "event");
            hip_check(hipEventCreate(&e1), "event");
            hip_check(hipEventRecord(e0, b->stream), "event");
            for (int r = 0; r < reps; ++r) {
                batch_order(b.get());
                batch_enqueue(b.get());
            }
            hip_check(hipEventRecord(e1, b->stream), "event");
            hip_check(hipEventSynchronize(e1), "event sync");
            float ms = 0.0f;
            hip_check(hipEventElapsedTime(&ms, e0, e1), "event time");
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            ms_out[k] = ms / reps;
        }
    });
}

int gpcg_solve_plain(gpcg_t h, int32_t n_out, const int32_t *outages, const double *rhs, double tol,
                     int32_t max_iter, double *x_out, double *flows_out, int32_t *iters_out, int32_t *status_out,
                     uint8_t *island_out, double *resid_out) {
    return guarded([&] {
        run_solve(h, 1, n_out, outages, rhs, tol, max_iter, x_out, flows_out, iters_out, status_out, island_out,
                  resid_out);
    });
}

int gpcg_get_order(gpcg_t h, int32_t n_out, int32_t *order) {
    return guarded([&] {
        if (!h || !order) fail(GPCG_E_ARG, "NULL argument");
        if (n_out != h->last_n_out) fail(GPCG_E_ARG, "n_out differs from the last solve");
        if (h->last_ordered) {
            std::vector<int32_t> sorted(n_out);
            hip_check(hipMemcpyAsync(sorted.data(), h->last_order, (size_t)n_out * sizeof(int32_t),
                                     hipMemcpyDeviceToHost, h->stream),
                      "copy");
            hip_check(hipStreamSynchronize(h->stream), "sync");
            for (int j = 0; j < n_out; ++j) order[j] = sorted[n_out - 1 - j];  // taken from the heavy end
        } else {
            for (int j = 0; j < n_out; ++j) order[j] = j;
        }
    });
}

int gpcg_get_sweeps(gpcg_t h, int32_t *waves, int64_t *wave_iterations) {
    return guarded([&] {
        if (!h || !waves || !wave_iterations) fail(GPCG_E_ARG, "NULL argument");
        unsigned long long n = 0;
        hip_check(hipMemcpyAsync(&n, h->sweeps.p, sizeof(n), hipMemcpyDeviceToHost, h->stream), "copy");
        hip_check(hipStreamSynchronize(h->stream), "sync");
        *waves = h->last_waves;
        *wave_iterations = (int64_t)n;
    });
}

int gpcg_set_timing(gpcg_t h, int enable) {
    return guarded([&] {
        if (!h) fail(GPCG_E_ARG, "NULL context");
        hip_check(hipSetDevice(h->device), "hipSetDevice");
        if (enable && !h->ev0) {
            hip_check(hipEventCreate(&h->ev0), "hipEventCreate");
            hip_check(hipEventCreate(&h->ev1), "hipEventCreate");
        }
        h->timing = enable != 0;
        h->timed = false;
    });
}

int gpcg_get_timing(gpcg_t h, double *pcg_ms) {
    return guarded([&] {
        if (!h || !pcg_ms) fail(GPCG_E_ARG, "NULL argument");
        if (!h->timed) fail(GPCG_E_ARG, "no timed solve yet (enable timing first)");
        hip_check(hipEventSynchronize(h->ev1), "hipEventSynchronize");
        float ms = 0.0f;
        hip_check(hipEventElapsedTime(&ms, h->ev0, h->ev1), "hipEventElapsedTime");
        *pcg_ms = ms;
    });
}

int gpcg_spmm(gpcg_t h, int32_t ncols, const int32_t *outages, const double *p, double *q, double *pq) {
    return guarded([&] {
        if (!h || !outages || !p || !q) fail(GPCG_E_ARG, "NULL argument");
        if (ncols <= 0 || ncols % h->S) fail(GPCG_E_ARG, "ncols must be a positive multiple of the block");
        hip_check(hipSetDevice(h->device), "hipSetDevice");
        // rows per chunk: the most, up to kSpmmMaxChunk, that the per-thread
        // staging takes and that keep the work-group's LDS in budget (with
        // narrow tiles the cap leaves room for more work-groups per CU)
        const int S = h->S, RS = 256 / S, nr = h->n_r, bw = h->bandwidth;
        const auto &rp = h->hA.rowptr;
        auto chunk_nnz = [&](int ch) {
            int mx = 0;
            for (int r0 = 0; r0 < nr; r0 += ch) mx = std::max(mx, rp[std::min(nr, r0 + ch)] - rp[r0]);
            return mx;
        };
        int ch = 0, max_nnz = 0;
        for (int c = (8192 / S) / RS * RS; c >= RS; c -= RS) {
            const int mx = chunk_nnz(c);
            if (!gpcg::spmm_chunk_fits(S, c, mx)) continue;
            ch = c;
            max_nnz = mx;
            if (c <= gpcg::kSpmmMaxChunk && gpcg::spmm_lds_bytes(S, bw, c, mx) <= gpcg::kSpmmLdsBudget) break;
        }
        if (ch == 0 || gpcg::spmm_lds_bytes(S, bw, ch, max_nnz) > 160 * 1024)
            fail(GPCG_E_UNSUPPORTED, "the matrix bandwidth is too large for the product's LDS window at this block");
        const int n_chunks = (nr + ch - 1) / ch;
        if (h->spmm_ch != ch) {  // lay A out per chunk (once per chunk height)
            std::vector<double> val((size_t)n_chunks * max_nnz, 0.0);
            std::vector<int32_t> col((size_t)n_chunks * max_nnz, 0), rpc((size_t)n_chunks * (ch + 1)),
                pre((size_t)n_chunks * ch, -1);
            for (int k = 0; k < n_chunks; ++k) {
                const int c0 = k * ch, c1 = std::min(nr, c0 + ch), base = std::max(0, c0 - bw), e0 = rp[c0];
                for (int e = e0; e < rp[c1]; ++e) {
                    val[(size_t)k * max_nnz + e - e0] = h->hA.val[e];
                    col[(size_t)k * max_nnz + e - e0] = h->hA.col[e] - base;
                }
                for (int t = 0; t <= ch; ++t) rpc[(size_t)k * (ch + 1) + t] = rp[std::min(c1, c0 + t)] - e0;
                for (int t = 0; t < ch && c0 + t < nr; ++t) pre[(size_t)k * ch + t] = h->h_prerow[c0 + t];
            }
            h->spmm_ch = 0;
            h->c_val.upload(val.data(), val.size(), h->stream);
            h->c_col.upload(col.data(), col.size(), h->stream);
            h->c_rp.upload(rpc.data(), rpc.size(), h->stream);
            h->c_pre.upload(pre.data(), pre.size(), h->stream);
            hip_check(hipStreamSynchronize(h->stream), "product layout upload");
            h->spmm_ch = ch;
            h->spmm_max_nnz = max_nnz;
        }
        gpcg::SpmmParams s{};
        s.n_r = nr;
        s.m = h->m;
        s.ncols = ncols;
        s.c_val = h->c_val.p;
        s.c_col = h->c_col.p;
        s.c_rp = h->c_rp.p;
        s.c_pre = h->c_pre.p;
        s.br_from = h->br_from.p;
        s.br_to = h->br_to.p;
        s.br_b = h->br_b.p;
        s.isl_lo = h->isl_lo.p;
        s.isl_hi = h->isl_hi.p;
        s.outages = outages;
        s.p = p;
        s.q = q;
        s.pq = pq;
        // Segment length: the grid runs in rounds of `slots` resident
        // work-groups (LDS-bound, at most four of 256 threads per CU), and a
        // work-group costs its chunks plus a prologue of about 2 bw rows;
        // take the length with the fewest chunk-times over all rounds.
        int cu = 256;
        (void)hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, h->device);
        const size_t lds = gpcg::spmm_lds_bytes(S, bw, ch, max_nnz);
        const long slots = (long)cu * std::max<long>(1, std::min<long>(4, (long)(160 * 1024) / (long)lds));
        const long tile_slots = ((ncols / S) + 7) / 8 * 8;  // the grid pads tiles to whole XCD rounds
        int nseg = 1;
        double best = 1e300;
        for (int cand = 1; cand <= n_chunks; ++cand) {
            const long segs = (n_chunks + cand - 1) / cand;
            if (cand > 1 && (n_chunks + cand - 2) / (cand - 1) == segs) continue;  // same split as cand - 1
            const long rounds = (tile_slots * segs + slots - 1) / slots;
            const double cost = (double)rounds * (cand + 2.0 * bw / ch);
            if (cost < best) {
                best = cost;
                nseg = cand;
            }
        }
        double *partial = nullptr;
        if (pq) {
            const size_t need = (size_t)((n_chunks + nseg - 1) / nseg) * ncols;
            if (h->partial.n < need) h->partial.alloc(need);
            partial = h->partial.p;
        }
        hip_check(gpcg::launch_spmm_partial(s, S, bw, ch, nseg, max_nnz, partial, h->stream), "spmm launch");
    });
}

}  // extern "C"
