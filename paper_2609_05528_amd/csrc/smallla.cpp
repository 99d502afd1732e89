// Small dense FP64 linear algebra on the host (n <= a few hundred): the
// one-sided Jacobi SVD (Hestenes), started from the eigenvectors of the
// Gram matrix, and the host thread pool.  Row-major storage.
#include <algorithm>
#include <cmath>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>

#include "dense.h"

namespace rtt {

// A pool of host worker threads (at most 15, started on first use and kept to the end of the
// process).  run(parts, f) calls f(0) .. f(parts - 1), each once, on the caller and the workers,
// and returns when all have finished.  A job lives on the caller's stack until every worker that
// picked it up has let it go.  Concurrent callers do not wait for each other: a caller that finds
// the pool busy does its parts alone, and so does a call made from inside a job of the pool.
class HostPool {
  public:
    static HostPool& get()
    {
        static HostPool* p = new HostPool();   // never destroyed: workers may still wait at exit
        return *p;
    }
    template <class F>
    void run(int parts, F&& f)
    {
        // a call from inside a job of the pool (nested) runs its parts in the calling thread
        if (parts <= 1 || nworkers_ == 0 || in_job()) {
            for (int i = 0; i < parts; ++i) f(i);
            return;
        }
        std::unique_lock<std::mutex> busy(run_m_, std::try_to_lock);
        if (!busy.owns_lock()) {
            for (int i = 0; i < parts; ++i) f(i);
            return;
        }
        Job j;
        j.f = [&f](int i) { f(i); };
        j.parts = parts;
        {
            std::lock_guard<std::mutex> lk(m_);
            cur_ = &j;
            ++gen_;
        }
        cv_.notify_all();
        work(j);
        while (j.done.load(std::memory_order_acquire) < parts) std::this_thread::yield();
        {
            std::lock_guard<std::mutex> lk(m_);
            cur_ = nullptr;
        }
        while (j.users.load(std::memory_order_acquire) > 0) std::this_thread::yield();
    }
    int threads() const { return nworkers_ + 1; }

  private:
    struct Job {
        std::function<void(int)> f;
        int parts = 0;
        std::atomic<int> next{0}, done{0}, users{0};
    };
    HostPool()
    {
        const int hw = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
        nworkers_ = hw - 1;
        for (int t = 0; t < nworkers_; ++t) std::thread([this] { loop(); }).detach();
    }
    static bool& in_job()
    {
        static thread_local bool v = false;
        return v;
    }
    static void work(Job& j)
    {
        bool& ij = in_job();
        const bool prev = ij;
        ij = true;
        for (;;) {
            const int i = j.next.fetch_add(1, std::memory_order_relaxed);
            if (i >= j.parts) break;
            j.f(i);
            j.done.fetch_add(1, std::memory_order_release);
        }
        ij = prev;
    }
    void loop()
    {
        uint64_t seen = 0;
        for (;;) {
            Job* j;
            {
                std::unique_lock<std::mutex> lk(m_);
                cv_.wait(lk, [&] { return gen_ != seen; });
                seen = gen_;
                j = cur_;
                if (!j) continue;
                j->users.fetch_add(1, std::memory_order_acq_rel);
            }
            work(*j);
            j->users.fetch_sub(1, std::memory_order_acq_rel);
        }
    }
    std::mutex run_m_, m_;
    std::condition_variable cv_;
    Job* cur_ = nullptr;
    uint64_t gen_ = 0;
    int nworkers_ = 0;
};

// f(lo, hi) over [0, n) split into contiguous parts, one per pool thread (parts of at least
// `grain` items).  The parts touch disjoint data, so the result does not depend on the split.
template <class F>
static void parallel_for(int n, int grain, F f)
{
    HostPool& pool = HostPool::get();
    const int parts = std::max(1, std::min(pool.threads(), n / std::max(1, grain)));
    if (parts == 1) {
        f(0, n);
        return;
    }
    pool.run(parts, [&](int t) { f((int)((int64_t)n * t / parts), (int)((int64_t)n * (t + 1) / parts)); });
}

void host_for(int n, const std::function<void(int)>& f)
{
    HostPool::get().run(n, [&f](int i) { f(i); });
}

// Eigenvectors of a symmetric n x n matrix S (row-major, destroyed): Householder reduction to
// tridiagonal form T = Q^T S Q with Q accumulated, then implicit symmetric QR steps with the
// Wilkinson shift on T (Golub and Van Loan, Matrix Computations, Sec. 8.3), the Givens rotations
// applied to the columns of Q.  On return row j of Zt (n x n, row-major) is eigenvector j: Q is
// kept transposed so that every update runs along contiguous memory.  The eigenvalues are not
// needed by the caller.
static void sym_eigvectors(std::vector<double>& S, int n, std::vector<double>& Zt)
{
    std::vector<double>& Z = Zt;
    Z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    std::vector<double> d(n, 0.0), e(n, 0.0), v(n), p(n), w(n), q(n);
    // reflector k: beta_k and v_k (length n - k - 1) kept for the back-transformation
    std::vector<double> hv((size_t)n * n, 0.0), hbeta(n, 0.0);
    auto A = [&](int i, int j) -> double& { return S[(size_t)i * n + j]; };
    // reduction: step k annihilates A[k+2:, k] with a reflector H = I - beta v v^T on rows k+1..
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;   // length of the active part
        double xn = 0.0;
        for (int i = 0; i < m; ++i) xn += A(k + 1 + i, k) * A(k + 1 + i, k);
        xn = std::sqrt(xn);
        const double x0 = A(k + 1, k);
        double beta = 0.0, alpha = x0;
        if (xn > 0.0) {
            alpha = x0 >= 0.0 ? -xn : xn;   // A[k+1,k] after the reflection
            // v = x - alpha e1 scaled so v[0] = 1
            const double v0 = x0 - alpha;
            v[0] = 1.0;
            for (int i = 1; i < m; ++i) v[i] = A(k + 1 + i, k) / v0;
            double vv = 0.0;
            for (int i = 0; i < m; ++i) vv += v[i] * v[i];
            beta = 2.0 / vv;
        }
        d[k] = A(k, k);
        e[k] = alpha;
        if (beta == 0.0) continue;
        // A22 <- H A22 H = A22 - v w^T - w v^T with p = beta A22 v, w = p - (beta/2)(p^T v) v
        // A22 is exactly symmetric (its updates add the same two products in either order), so
        // A22 v is summed along contiguous rows: the same terms in the same order per entry.
        std::fill(q.begin(), q.begin() + m, 0.0);
        for (int j = 0; j < m; ++j) {
            const double vj = v[j];
            const double* aj = &A(k + 1 + j, k + 1);
            for (int i = 0; i < m; ++i) q[i] += vj * aj[i];
        }
        double pv = 0.0;
        for (int i = 0; i < m; ++i) {
            p[i] = beta * q[i];
            pv += p[i] * v[i];
        }
        for (int i = 0; i < m; ++i) w[i] = p[i] - 0.5 * beta * pv * v[i];
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) A(k + 1 + i, k + 1 + j) -= v[i] * w[j] + w[i] * v[j];
        hbeta[k] = beta;
        std::copy(v.begin(), v.begin() + m, hv.begin() + (size_t)k * n);
    }
    if (n >= 2) {
        d[n - 2] = A(n - 2, n - 2);
        e[n - 2] = A(n - 1, n - 2);
    }
    d[n - 1] = A(n - 1, n - 1);
    e[n - 1] = 0.0;
    // implicit QR on the tridiagonal (d, e): e[i] couples i and i+1.  The rotations are recorded.
    // Q (the reflectors, then the rotations, in order) is formed afterwards, a range of columns of
    // Qt at a time: every column sees the same updates in the same order.
    struct Rot {
        int k;
        double c, s;
    };
    std::vector<Rot> rots;
    rots.reserve((size_t)8 * n * n);
    const double eps = 2.3e-16;
    int hi = n - 1, guard = 0;
    while (hi > 0 && guard < 64 * n) {
        // deflate converged off-diagonals at the bottom
        if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
            e[hi - 1] = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
        if (lo > 0) e[lo - 1] = 0.0;
        ++guard;
        // Wilkinson shift from the trailing 2 x 2 block of [lo, hi]
        const double dd = 0.5 * (d[hi - 1] - d[hi]);
        const double eh = e[hi - 1];
        const double mu = d[hi] - eh * eh / (dd + (dd >= 0.0 ? 1.0 : -1.0) * std::hypot(dd, eh));
        double x = d[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            // rotation in the plane (k, k+1) that zeroes z against x
            const double r = std::hypot(x, z);
            const double c = r > 0.0 ? x / r : 1.0, sn = r > 0.0 ? z / r : 0.0;
            if (k > lo) e[k - 1] = r;
            const double a = d[k], b = e[k], d2 = d[k + 1];
            d[k] = c * c * a + 2.0 * c * sn * b + sn * sn * d2;
            d[k + 1] = sn * sn * a - 2.0 * c * sn * b + c * c * d2;
            e[k] = c * sn * (d2 - a) + (c * c - sn * sn) * b;
            if (k + 1 < hi) {
                z = sn * e[k + 1];   // bulge at (k+2, k)
                e[k + 1] *= c;
                x = e[k];
            }
            rots.push_back({k, c, sn});
        }
    }
    // one contiguous range of columns of Qt per host thread, worked on in a private copy (no
    // cache line is shared between threads while the updates run)
    parallel_for(n, 8, [&](int r0, int r1) {
        const int w = r1 - r0;
        std::vector<double> L((size_t)n * w), ql(w);
        for (int i = 0; i < n; ++i) std::copy(&Z[(size_t)i * n + r0], &Z[(size_t)i * n + r1], &L[(size_t)i * w]);
        // Q <- Q H_k on columns k+1.. (rows k+1.. of Qt), k ascending
        for (int k = 0; k + 2 < n; ++k) {
            const double beta = hbeta[k];
            if (beta == 0.0) continue;
            const int m = n - k - 1;
            const double* vk = &hv[(size_t)k * n];
            std::fill(ql.begin(), ql.end(), 0.0);
            for (int j = 0; j < m; ++j) {
                const double* zj = &L[(size_t)(k + 1 + j) * w];
                for (int r2 = 0; r2 < w; ++r2) ql[r2] += zj[r2] * vk[j];
            }
            for (int j = 0; j < m; ++j) {
                double* zj = &L[(size_t)(k + 1 + j) * w];
                const double bv = beta * vk[j];
                for (int r2 = 0; r2 < w; ++r2) zj[r2] -= ql[r2] * bv;
            }
        }
        for (const Rot& g : rots) {
            double* zk = &L[(size_t)g.k * w];
            double* zk1 = zk + w;
            const double c = g.c, sn = g.s;
            for (int r2 = 0; r2 < w; ++r2) {
                const double u0 = zk[r2], u1 = zk1[r2];
                zk[r2] = c * u0 + sn * u1;
                zk1[r2] = -sn * u0 + c * u1;
            }
        }
        for (int i = 0; i < n; ++i) std::copy(&L[(size_t)i * w], &L[(size_t)(i + 1) * w], &Z[(size_t)i * n + r0]);
    });
}

// <a, b> with eight partial sums (a fixed order, vectorisable)
static double dot8(const double* a, const double* b, int n)
{
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int i = 0;
    for (; i + 8 <= n; i += 8)
        for (int u = 0; u < 8; ++u) s[u] += a[i + u] * b[i + u];
    for (; i < n; ++i) s[i & 7] += a[i] * b[i];
    return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

void jacobi_svd(const std::vector<double>& M, int n, std::vector<double>& U, std::vector<double>& s,
                std::vector<double>& W)
{
    // work on columns: a[j] = column j of the working matrix (contiguous), v[j] = column j of W.
    // The sweeps start from M Z, Z the eigenvectors of M^T M: its columns are already nearly
    // orthogonal, so the one-sided Jacobi that follows (and sets the accuracy) needs few sweeps.
    std::vector<double> a((size_t)n * n, 0.0), v((size_t)n * n, 0.0);
    {
        std::vector<double> G((size_t)n * n, 0.0), Z;
        parallel_for(n, 16, [&](int i0, int i1) {
            for (int k = 0; k < n; ++k) {
                const double* mk = &M[(size_t)k * n];
                for (int i = i0; i < i1; ++i) {
                    const double mi = mk[i];
                    if (mi == 0.0) continue;
                    double* gi = &G[(size_t)i * n];
                    for (int j = 0; j < n; ++j) gi[j] += mi * mk[j];
                }
            }
        });
        sym_eigvectors(G, n, Z);   // row j of Z: eigenvector j
        v = Z;
        // a[j] = M z_j, accumulated along rows of M^T
        std::vector<double> Mt((size_t)n * n);
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) Mt[(size_t)k * n + i] = M[(size_t)i * n + k];
        parallel_for(n, 16, [&](int j0, int j1) {
            for (int j = j0; j < j1; ++j) {
                const double* zj = &v[(size_t)j * n];
                double* aj = &a[(size_t)j * n];
                for (int k = 0; k < n; ++k) {
                    const double z = zj[k];
                    if (z == 0.0) continue;
                    const double* mk = &Mt[(size_t)k * n];
                    for (int i = 0; i < n; ++i) aj[i] += z * mk[i];
                }
            }
        });
    }
    std::vector<double> nrm(n);
    for (int j = 0; j < n; ++j) nrm[j] = dot8(&a[(size_t)j * n], &a[(size_t)j * n], n);
    const double eps = 1e-15;
    // one rotation of columns p < q; returns 1 if it was needed
    auto rotate = [&](int p, int q) -> int {
        double* ap = &a[(size_t)p * n];
        double* aq = &a[(size_t)q * n];
        const double g = dot8(ap, aq, n);
        const double al = nrm[p], be = nrm[q];
        if (std::fabs(g) <= eps * std::sqrt(al * be) || g == 0.0) return 0;
        const double zeta = (be - al) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        for (int i = 0; i < n; ++i) {
            const double x = ap[i], y = aq[i];
            ap[i] = c * x - sn * y;
            aq[i] = sn * x + c * y;
        }
        nrm[p] = dot8(ap, ap, n);
        nrm[q] = dot8(aq, aq, n);
        double* vp = &v[(size_t)p * n];
        double* vq = &v[(size_t)q * n];
        for (int i = 0; i < n; ++i) {
            const double x = vp[i], y = vq[i];
            vp[i] = c * x - sn * y;
            vq[i] = sn * x + c * y;
        }
        return 1;
    };
    // Sweeps in block round-robin order: the columns form NB blocks; in round r of a sweep the
    // blocks meet in NB/2 disjoint pairs (the circle method), and each pair rotates every column
    // of one block against every column of the other, the pairs inside each block in the first
    // round.  Every pair of columns is visited once per sweep.  The pairs of a round touch
    // disjoint columns and run on separate host threads; NB is fixed, so the result does not
    // depend on the number of threads.
    constexpr int NB = 16, NP = NB / 2, NR = NB - 1, MAX_SWEEPS = 60;
    auto blk = [n](int b) { return (int)((int64_t)n * b / NB); };
    auto pair_task = [&](int r, int t) {
        int P = t == 0 ? r : (r + t) % NR;
        int Q = t == 0 ? NB - 1 : (r - t + NR) % NR;
        if (P > Q) std::swap(P, Q);
        int cnt = 0;
        if (r == 0)
            for (int B : {P, Q})
                for (int p = blk(B); p < blk(B + 1); ++p)
                    for (int q = p + 1; q < blk(B + 1); ++q) cnt += rotate(p, q);
        for (int p = blk(P); p < blk(P + 1); ++p)
            for (int q = blk(Q); q < blk(Q + 1); ++q) cnt += rotate(p, q);
        return cnt;
    };
    // All sweeps run inside one job of the host pool: the participants take the pairs of a round
    // from a counter and wait (spinning) until every pair of the round is done before the next
    // round, instead of one pool job per round.  A participant that starts late, or alone (the
    // pool busy or nested), finds the taken pairs done or takes them itself, so nothing waits for a
    // thread that is not running.  Every participant sums the same per-pair rotation counts and
    // stops after the same sweep.
    std::unique_ptr<std::atomic<int>[]> next(new std::atomic<int>[MAX_SWEEPS * NR]),
        done(new std::atomic<int>[MAX_SWEEPS * NR]);
    for (int i = 0; i < MAX_SWEEPS * NR; ++i) {
        next[i].store(0, std::memory_order_relaxed);
        done[i].store(0, std::memory_order_relaxed);
    }
    std::vector<int> cnt((size_t)MAX_SWEEPS * NR * NP, 0);
    auto participant = [&]() {
        for (int sweep = 0; sweep < MAX_SWEEPS; ++sweep) {
            for (int r = 0; r < NR; ++r) {
                const int id = sweep * NR + r;
                for (;;) {
                    const int t = next[id].fetch_add(1, std::memory_order_relaxed);
                    if (t >= NP) break;
                    cnt[(size_t)id * NP + t] = pair_task(r, t);
                    done[id].fetch_add(1, std::memory_order_release);
                }
                while (done[id].load(std::memory_order_acquire) < NP) std::this_thread::yield();
            }
            int rot = 0;
            for (size_t i = (size_t)sweep * NR * NP; i < (size_t)(sweep + 1) * NR * NP; ++i) rot += cnt[i];
            if (rot == 0) return;
        }
    };
    const int parts = n >= 128 ? std::min(HostPool::get().threads(), NP) : 1;
    if (parts == 1)
        participant();
    else
        HostPool::get().run(parts, [&](int) { participant(); });
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::vector<double> sv(n);
    for (int j = 0; j < n; ++j) sv[j] = std::sqrt(dot8(&a[(size_t)j * n], &a[(size_t)j * n], n));
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return sv[x] > sv[y]; });
    U.assign((size_t)n * n, 0.0);
    W.assign((size_t)n * n, 0.0);
    s.assign(n, 0.0);
    for (int jj = 0; jj < n; ++jj) {
        const int j = ord[jj];
        s[jj] = sv[j];
        for (int i = 0; i < n; ++i) {
            U[(size_t)i * n + jj] = sv[j] > 0.0 ? a[(size_t)j * n + i] / sv[j] : 0.0;
            W[(size_t)i * n + jj] = v[(size_t)j * n + i];
        }
    }
}

}  // namespace rtt
