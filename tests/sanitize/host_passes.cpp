// The library's host-side preparation passes (assembly, reverse
// Cuthill-McKee, ILU(0), topology) driven through the C ABI on seeded random
// grids and on malformed inputs, for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code.  Prints "ok" and exits 0 when
// every call behaved; the sanitizers abort on any memory or UB error.
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <random>
#include <vector>

#include "gpcg.h"

static int fails = 0;
#define CHECK(c)                                                    \
    do {                                                            \
        if (!(c)) {                                                 \
            std::printf("check failed line %d: %s\n", __LINE__, #c); \
            ++fails;                                                \
        }                                                           \
    } while (0)

int main() {
    std::mt19937 rng(12345);
    for (int trial = 0; trial < 300; ++trial) {
        const int n = 2 + (int)(rng() % 80);
        std::vector<int32_t> f, t;
        for (int v = 1; v < n; ++v) {  // a random spanning tree, then extra branches (parallel ones allowed)
            f.push_back((int32_t)(rng() % v));
            t.push_back(v);
        }
        const int extra = (int)(rng() % (n + 1));
        for (int k = 0; k < extra; ++k) {
            const int a = (int)(rng() % n), b = (int)(rng() % n);
            if (a == b) continue;
            f.push_back(a);
            t.push_back(b);
        }
        const int m = (int)f.size();
        std::vector<double> x(m), sh(n);
        for (auto &v : x) v = 0.01 + (rng() % 1000) * 3e-4;
        for (auto &v : sh) v = (rng() % 100) * 5e-4;
        std::vector<int32_t> perm(n - 1);
        CHECK(gpcg_rcm(n, m, f.data(), t.data(), perm.data()) == GPCG_OK);
        std::vector<int> seen(n, 0);
        for (int b : perm) {
            CHECK(b >= 1 && b < n);
            if (b >= 1 && b < n) ++seen[b];
        }
        for (int b = 1; b < n; ++b) CHECK(seen[b] == 1);
        const int cap = n - 1 + 2 * m;
        std::vector<int32_t> rp(n), col(cap);
        std::vector<double> val(cap);
        int32_t nnz = 0;
        for (int variant = 0; variant < 3; ++variant) {
            const double *shp = variant == 2 ? sh.data() : nullptr;
            const int32_t *pp = variant >= 1 ? perm.data() : nullptr;
            CHECK(gpcg_assemble(n, m, f.data(), t.data(), x.data(), shp, pp, rp.data(), col.data(), val.data(), cap,
                                &nnz) == GPCG_OK);
            gpcg_csr A{n - 1, nnz, rp.data(), col.data(), val.data()};
            std::vector<int32_t> lr(n), lc(nnz + 1), ur(n), uc(nnz + 1);
            std::vector<double> lv(nnz + 1), uv(nnz + 1);
            int32_t nl = 0, nu = 0;
            CHECK(gpcg_ilu0(&A, lr.data(), lc.data(), lv.data(), &nl, ur.data(), uc.data(), uv.data(), &nu) ==
                  GPCG_OK);
            CHECK(nl + nu == nnz);
        }
        std::vector<uint8_t> br(m);
        std::vector<int32_t> pre(n), sub(n), lo(m), hi(m);
        CHECK(gpcg_topology(n, m, f.data(), t.data(), br.data(), pre.data(), sub.data(), lo.data(), hi.data()) ==
              GPCG_OK);
        CHECK(sub[0] == n);
        // malformed inputs: each must return an error code, never crash
        std::vector<int32_t> bad = perm;
        if (n > 2) {
            bad[0] = bad[1];
            CHECK(gpcg_assemble(n, m, f.data(), t.data(), x.data(), nullptr, bad.data(), rp.data(), col.data(),
                                val.data(), cap, &nnz) == GPCG_E_ARG);
        }
        CHECK(gpcg_assemble(n, m, f.data(), t.data(), x.data(), nullptr, nullptr, rp.data(), col.data(), val.data(),
                            0, &nnz) == GPCG_E_ARG);
        std::vector<int32_t> f2 = f;
        f2[0] = n;  // out of range
        CHECK(gpcg_rcm(n, m, f2.data(), t.data(), perm.data()) == GPCG_E_ARG);
        CHECK(gpcg_topology(n, m, f2.data(), t.data(), br.data(), pre.data(), sub.data(), lo.data(), hi.data()) ==
              GPCG_E_ARG);
    }
    // a disconnected grid, a CSR without a diagonal, NULL pointers
    {
        const int32_t f[] = {0, 2}, t[] = {1, 3};
        std::vector<uint8_t> br(2);
        std::vector<int32_t> pre(4), sub(4), lo(2), hi(2);
        CHECK(gpcg_topology(4, 2, f, t, br.data(), pre.data(), sub.data(), lo.data(), hi.data()) == GPCG_E_ARG);
        const int32_t rp[] = {0, 1, 2}, cl[] = {1, 0};
        const double v[] = {1.0, 1.0};
        gpcg_csr A{2, 2, rp, cl, v};
        int32_t o[3], c[3], nl, nu;
        double d[3];
        CHECK(gpcg_ilu0(&A, o, c, d, &nl, o, c, d, &nu) == GPCG_E_PATTERN);
        CHECK(gpcg_ilu0(nullptr, o, c, d, &nl, o, c, d, &nu) == GPCG_E_ARG);
        CHECK(gpcg_rcm(2, 1, f, t, nullptr) == GPCG_E_ARG);
    }
    std::printf(fails ? "FAILED %d\n" : "ok\n", fails);
    return fails ? 1 : 0;
}
