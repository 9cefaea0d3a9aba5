// Captured mat-vecs and batches of plans.
//
// A mat-vec is a fixed sequence of kernel launches (gather, P2P, S2M, M2M,
// M2L, L2L, L2T, scatter, corrections) whose arguments depend only on the
// plan, the operator and the two vectors.  graph_matvec captures it once per
// (operator, input, output) into a HIP graph and replays it, so a GMRES step
// costs one graph launch instead of dozens of kernel launches.
//
// A batch holds many plans (instances of different size and wavenumber on
// the same device).  fda_batch_matvec captures every instance's mat-vec into
// ONE graph, each instance on one of several forked capture streams, so a
// single launch runs all instances concurrently and fills the device even
// when each instance alone is small.  fda_batch_solve runs the instances'
// GMRES solves from a pool of host threads, each on its own stream, every
// step through its plan's captured mat-vec.
//
// Graphs contain kernel nodes and event waits only (no memset nodes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <functional>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "device.hpp"

namespace fdbem {

#define HIP_CHECK(expr)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            throw std::runtime_error(std::string("HIP error ") + hipGetErrorString(e_) + " at " + \
                                     __FILE__ + ":" + std::to_string(__LINE__));                 \
    } while (0)

constexpr size_t kGraphCache = 8;

static hipGraphExec_t capture(hipStream_t cap, const std::function<void(hipStream_t)> &body)
{
    HIP_CHECK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    try {
        body(cap);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(cap, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    hipGraph_t g = nullptr;
    HIP_CHECK(hipStreamEndCapture(cap, &g));
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_CHECK(e);
    return exec;
}

void graph_matvec(Plan &P, int op, const double2 *in, double2 *out, hipStream_t st)
{
    Device &D = *P.dev;
    if (!D.use_graph || D.timing) {
        device_matvec(P, op, in, out, st);
        return;
    }
    auto it = std::find_if(D.graphs.begin(), D.graphs.end(), [&](const Device::GraphEntry &e) {
        return e.op == op && e.in == in && e.out == out;
    });
    if (it == D.graphs.end()) {
        if (!D.cap) HIP_CHECK(hipStreamCreateWithFlags(&D.cap, hipStreamNonBlocking));
        if (D.graphs.size() >= kGraphCache) {
            (void)hipGraphExecDestroy(D.graphs.front().exec);
            D.graphs.erase(D.graphs.begin());
        }
        Device::GraphEntry e;
        e.op = op;
        e.in = in;
        e.out = out;
        e.exec = capture(D.cap, [&](hipStream_t s) { device_matvec(P, op, in, out, s); });
        D.graphs.push_back(e);
        it = D.graphs.end() - 1;
    }
    HIP_CHECK(hipGraphLaunch(it->exec, st));
}

void graph_release(Device &D)
{
    for (auto &e : D.graphs)
        if (e.exec) (void)hipGraphExecDestroy(e.exec);
    D.graphs.clear();
    if (D.cap) (void)hipStreamDestroy(D.cap);
    D.cap = nullptr;
}

// ---------------------------------------------------------------- batches
struct Batch {
    std::vector<Plan *> plans;
    int device = 0;
    std::vector<hipStream_t> branch;   // forked capture streams
    hipStream_t cap = nullptr;
    std::vector<hipEvent_t> ev;        // fork + one join per branch
    hipGraphExec_t exec = nullptr;
    int op = -1;
    std::vector<const void *> in;
    std::vector<void *> out;
};

static constexpr int kBranches = 16;

Batch *batch_create(Plan *const *plans, int n)
{
    Batch *B = new Batch();
    try {
        B->plans.assign(plans, plans + n);
        B->device = plans[0]->dev->device;
        for (Plan *p : B->plans)
            if (p->dev->device != B->device) throw std::invalid_argument("batch plans live on different devices");
        HIP_CHECK(hipSetDevice(B->device));
        HIP_CHECK(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
        const int nb = std::min(n, kBranches);
        B->branch.resize(nb, nullptr);
        for (auto &s : B->branch) HIP_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        B->ev.resize(nb + 1, nullptr);
        for (auto &e : B->ev) HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    } catch (...) {
        batch_destroy(B);
        throw;
    }
    return B;
}

void batch_destroy(Batch *B)
{
    if (!B) return;
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    for (auto s : B->branch)
        if (s) (void)hipStreamDestroy(s);
    if (B->cap) (void)hipStreamDestroy(B->cap);
    for (auto e : B->ev)
        if (e) (void)hipEventDestroy(e);
    delete B;
}

void batch_matvec(Batch *B, int op, const double2 *const *in, double2 *const *out, hipStream_t st)
{
    const int n = (int)B->plans.size();
    bool same = B->exec && B->op == op;
    for (int i = 0; same && i < n; ++i) same = B->in[i] == in[i] && B->out[i] == out[i];
    if (!same) {
        if (B->exec) (void)hipGraphExecDestroy(B->exec);
        B->exec = nullptr;
        const int nb = (int)B->branch.size();
        B->exec = capture(B->cap, [&](hipStream_t s) {
            HIP_CHECK(hipEventRecord(B->ev[0], s));
            for (int b = 0; b < nb; ++b) HIP_CHECK(hipStreamWaitEvent(B->branch[b], B->ev[0], 0));
            // largest instances first so the branches finish together
            std::vector<int> order(n);
            for (int i = 0; i < n; ++i) order[i] = i;
            std::stable_sort(order.begin(), order.end(),
                             [&](int a, int b) { return B->plans[a]->N > B->plans[b]->N; });
            std::vector<int64_t> load(nb, 0);
            for (int i : order) {
                const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                load[b] += B->plans[i]->N;
                device_matvec(*B->plans[i], op, in[i], out[i], B->branch[b]);
            }
            for (int b = 0; b < nb; ++b) {
                HIP_CHECK(hipEventRecord(B->ev[b + 1], B->branch[b]));
                HIP_CHECK(hipStreamWaitEvent(s, B->ev[b + 1], 0));
            }
        });
        B->op = op;
        B->in.assign(in, in + n);
        B->out.assign(out, out + n);
    }
    HIP_CHECK(hipGraphLaunch(B->exec, st));
}

// GMRES for every instance; returns the number of instances that did not converge
int batch_solve(Batch *B, int op, const double2 *const *rhs, double tol, int maxit, int restart, int precond,
                double2 *const *x, int *iters, double *relres, int *status)
{
    const int n = (int)B->plans.size();
    // preconditioner set-up (synchronous HIP calls) before the threads start capturing
    for (Plan *p : B->plans) {
        if (precond && !p->dev->bj.inv) build_block_jacobi(*p, *p->dev);
        if (precond == 3) learned_targets(*p);
    }
    const int nt = std::max(1, std::min(n, (int)std::thread::hardware_concurrency() > 0
                                               ? std::min(16, (int)std::thread::hardware_concurrency())
                                               : 4));
    std::atomic<int> next(0);
    std::vector<std::string> errors(nt);
    auto worker = [&](int t) {
        hipStream_t st = nullptr;
        try {
            HIP_CHECK(hipSetDevice(B->device));
            HIP_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            for (int i = next++; i < n; i = next++) {
                Plan &P = *B->plans[i];
                const int saved = P.dev->use_graph;
                P.dev->use_graph = 1;
                int it = 0;
                double rr = 0;
                int rc;
                try {
                    rc = device_gmres(P, op, rhs[i], tol, maxit, restart, precond, x[i], &it, &rr, nullptr, st);
                } catch (...) {
                    P.dev->use_graph = saved;
                    throw;
                }
                P.dev->use_graph = saved;
                if (iters) iters[i] = it;
                if (relres) relres[i] = rr;
                if (status) status[i] = rc;
            }
            HIP_CHECK(hipStreamSynchronize(st));
        } catch (const std::exception &e) {
            errors[t] = e.what();
        }
        if (st) (void)hipStreamDestroy(st);
    };
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t) pool.emplace_back(worker, t);
    for (auto &th : pool) th.join();
    for (const auto &e : errors)
        if (!e.empty()) throw std::runtime_error(e);
    int bad = 0;
    if (status)
        for (int i = 0; i < n; ++i) bad += status[i] != 0;
    return bad;
}

}  // namespace fdbem
