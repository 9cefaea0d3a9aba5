// C ABI of the library (declared in include/fdbem.h).  Every entry point
// catches exceptions and turns them into status codes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fdbem.h"
#include "device.hpp"

namespace fdbem {
Plan *plan_create_host(int64_t n, const double *pts, const double *nrm, const double *w, int64_t n_elem,
                       const double *elem, double k, double eps, const Options &opt);
std::string plan_stats(const Plan &P);
}  // namespace fdbem

using namespace fdbem;

struct fda_plan {
    Plan *P;
};

struct fda_net {
    LearnedNet *N;
};

struct fda_batch {
    Batch *B;
    std::vector<fda_plan *> plans;
};

static thread_local std::string g_err;

static int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

template <typename F>
static int guarded(F &&f)
{
    try {
        g_err.clear();
        return f();
    } catch (const std::invalid_argument &e) {
        return fail(FDA_EINVAL, e.what());
    } catch (const std::bad_alloc &e) {
        return fail(FDA_ENOMEM, "out of host memory");
    } catch (const std::runtime_error &e) {
        const std::string m = e.what();
        if (m.find("hipErrorOutOfMemory") != std::string::npos || m.find("out of memory") != std::string::npos)
            return fail(FDA_ENOMEM, m);
        if (m.find("HIP error") != std::string::npos) return fail(FDA_EHIP, m);
        return fail(FDA_ENOTSUP, m);
    } catch (...) {
        return fail(FDA_EHIP, "unknown error");
    }
}

extern "C" {

int fda_default_opts(fda_opts *o)
{
    if (!o) return fail(FDA_EINVAL, "null options");
    Options d;
    o->svd_eps = 0;
    o->lowrank_eps = 0;
    o->leaf_cap = d.leaf_cap;
    o->leaf_rule = d.leaf_rule;
    o->c_d = d.c_d;
    o->far_field = d.far_field;
    o->lf_grid = 0;
    o->precision = FDA_PREC_FP64;
    o->corrections = 1;
    o->verbose = 0;
    o->wedge_factor = d.wedge_factor;
    o->m2l_tile = 0;
    o->p2p_threshold = 0;
    o->coupling = 1.0;
    o->autotune = 1;
    o->slab_mb = 0;
    o->hf_template = 0;
    o->original = 0;
    o->serial_slabs = 0;
    o->chunk_kernel = 0;
    return FDA_OK;
}

int bem_nystrom_nodes(int64_t n_elem, const double *elem, double *pts, double *nrm, double *w)
{
    return guarded([&] {
        if (n_elem <= 0 || !elem || !pts || !nrm || !w) throw std::invalid_argument("bad nystrom arguments");
        nystrom_nodes(n_elem, elem, pts, nrm, w);
        return FDA_OK;
    });
}

int bem_near_correction(int64_t n_elem, const double *elem, const double *pts, const double *nrm, const double *w,
                        double k, int op, double coupling, int64_t *nnz_out, int64_t *row_ptr, int64_t *col,
                        double *val)
{
    return guarded([&] {
        if (n_elem <= 0 || !elem || !pts || !nrm || !w || !nnz_out) throw std::invalid_argument("null argument");
        if (!(k > 0) || !std::isfinite(k)) throw std::invalid_argument("wavenumber must be positive");
        if (op != FDA_OP_BM_H && op != FDA_OP_BM_G) throw std::invalid_argument("op must be FDA_OP_BM_H or FDA_OP_BM_G");
        if (!std::isfinite(coupling)) throw std::invalid_argument("non-finite coupling");
        std::vector<int64_t> rp, cl;
        std::vector<cplx> vl;
        correction_table_host(n_elem, elem, pts, nrm, w, k, op, coupling != 0 ? coupling : 1.0, rp, cl, vl);
        *nnz_out = (int64_t)cl.size();
        if (row_ptr && col && val) {
            std::memcpy(row_ptr, rp.data(), sizeof(int64_t) * rp.size());
            std::memcpy(col, cl.data(), sizeof(int64_t) * cl.size());
            std::memcpy(val, vl.data(), sizeof(cplx) * vl.size());
        }
        return FDA_OK;
    });
}

// Options of the C ABI in the internal form (NULL: defaults), validated.
static Options parse_opts(const fda_opts *o)
{
    Options opt;
    if (o) {
        opt.svd_eps = o->svd_eps;
        opt.lowrank_eps = o->lowrank_eps;
        opt.leaf_cap = o->leaf_cap > 0 ? o->leaf_cap : 64;
        opt.leaf_rule = o->leaf_rule;
        opt.c_d = o->c_d > 0 ? o->c_d : opt.c_d;
        opt.far_field = o->far_field;
        opt.lf_grid = o->lf_grid;
        opt.precision = o->precision;
        opt.corrections = o->corrections;
        opt.verbose = o->verbose;
        opt.wedge_factor = o->wedge_factor > 0 ? o->wedge_factor : opt.wedge_factor;
        opt.m2l_tile = o->m2l_tile;
        if (o->p2p_threshold != 0) opt.p2p_threshold = o->p2p_threshold;
        if (!std::isfinite(o->coupling)) throw std::invalid_argument("non-finite coupling");
        opt.coupling = o->coupling != 0 ? o->coupling : 1.0;
        opt.autotune = o->autotune;
        if (o->slab_mb < 0) throw std::invalid_argument("negative slab size");
        if (o->slab_mb > 0) opt.slab_mb = o->slab_mb;
        if (o->hf_template < 0 || o->hf_template > 1) throw std::invalid_argument("unknown high-frequency template rule");
        opt.hf_template = o->hf_template;
        if (o->original < 0 || o->original > 1) throw std::invalid_argument("original must be 0 or 1");
        opt.original = o->original;
        opt.serial_slabs = o->serial_slabs ? 1 : 0;
        if (o->chunk_kernel < 0 || o->chunk_kernel > 1) throw std::invalid_argument("chunk_kernel must be 0 or 1");
        opt.chunk_kernel = o->chunk_kernel;
    }
    if (opt.precision < FDA_PREC_FP64 || opt.precision > FDA_PREC_BOTH) throw std::invalid_argument("unknown precision");
    if (opt.leaf_rule != 0) throw std::invalid_argument("unknown leaf rule");
    return opt;
}

int fda_analyze(const fda_geometry *g, double k, double eps, const fda_opts *o, char *buf, size_t len)
{
    return guarded([&] {
        if (!g || !buf) throw std::invalid_argument("null geometry or buffer");
        const Options opt = parse_opts(o);
        std::unique_ptr<Plan> P(plan_create_host(g->n_nodes, g->pts, g->nrm, g->w, g->n_elem, g->elem, k, eps, opt));
        const std::string s = plan_stats(*P);
        if (s.size() + 1 > len) throw std::invalid_argument("stats buffer too small");
        std::memcpy(buf, s.c_str(), s.size() + 1);
        return FDA_OK;
    });
}

int fda_build(const fda_geometry *g, double k, double eps, const fda_opts *o, fda_plan **out)
{
    return guarded([&] {
        if (!g || !out) throw std::invalid_argument("null geometry or output pointer");
        *out = nullptr;
        const Options opt = parse_opts(o);
        Plan *P = plan_create_host(g->n_nodes, g->pts, g->nrm, g->w, g->n_elem, g->elem, k, eps, opt);
        try {
            device_upload(*P);
        } catch (...) {
            device_free(*P);
            delete P;
            throw;
        }
        fda_plan *h = new fda_plan{P};
        *out = h;
        return FDA_OK;
    });
}

// Operator code valid for this plan: a known base operator, no bits beyond
// FDA_OP_FP32, an FP32 far field only on plans that hold one, and the
// corrected operators only with their correction tables.
static void check_op(const Plan &P, int op)
{
    const int base = op & 0xff;
    if (base < FDA_OP_RAW_H || base > FDA_OP_BM_G || (op & ~0x1ff)) throw std::invalid_argument("unknown operator");
    if ((op & FDA_OP_FP32) && P.opt.precision == FDA_PREC_FP64)
        throw std::invalid_argument("FP32 operator requested on an FP64-only plan");
    if (base == FDA_OP_BM_H && !P.has_corr)
        throw std::invalid_argument("the corrected H operator needs a plan built with elements");
    if (base == FDA_OP_BM_G && !P.has_corr_g)
        throw std::invalid_argument("the corrected G operator needs a plan built with elements and corrections & 2");
}

int fda_matvec(fda_plan *plan, int op, const void *in_dev, void *out_dev, void *stream)
{
    return guarded([&] {
        if (!plan || !in_dev || !out_dev) throw std::invalid_argument("null argument");
        if (in_dev == out_dev) throw std::invalid_argument("input and output must not alias");
        Plan &P = *plan->P;
        check_op(P, op);
        // replays a captured graph when the plan has graphs on (fda_set_graph)
        graph_matvec(P, op, (const double2 *)in_dev, (double2 *)out_dev, (hipStream_t)stream);
        return FDA_OK;
    });
}

int fda_matvec_noalloc(fda_plan *plan, int op, const void *in_dev, void *out_dev, void *stream)
{
    return guarded([&] {
        if (!plan || !in_dev || !out_dev) throw std::invalid_argument("null argument");
        if (in_dev == out_dev) throw std::invalid_argument("input and output must not alias");
        Plan &P = *plan->P;
        check_op(P, op);
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != P.dev->device)
            throw std::invalid_argument("the plan's device is not the current device");
        device_matvec_static(P, op, (const double2 *)in_dev, (double2 *)out_dev, (hipStream_t)stream);
        return FDA_OK;
    });
}

int bm_solve(fda_plan *plan, int op, const void *rhs_dev, double tol, int maxit, int restart, int precond,
             void *x_dev, int *iters_out, double *relres_out, double *resid_hist, void *stream)
{
    return guarded([&] {
        if (!plan || !rhs_dev || !x_dev) throw std::invalid_argument("null argument");
        if (!(tol > 0) || maxit < 1 || restart < 1) throw std::invalid_argument("bad solver parameters");
        if (precond < 0 || precond > 3) throw std::invalid_argument("unknown preconditioner");
        Plan &P = *plan->P;
        check_op(P, op);
        const int rc = device_gmres(P, op, (const double2 *)rhs_dev, tol, maxit, restart, precond, (double2 *)x_dev,
                                    iters_out, relres_out, resid_hist, (hipStream_t)stream);
        if (rc == FDA_NOT_CONVERGED) return fail(rc, "GMRES did not reach the tolerance");
        if (rc == FDA_NONFINITE) return fail(rc, "non-finite value in GMRES");
        if (rc == FDA_EBREAKDOWN) return fail(rc, "GMRES breakdown");
        if (rc == FDA_ENOTSUP) return fail(rc, "preconditioner not available (1 and 3 need elements, 2 loaded factors)");
        return rc;
    });
}

int fda_rhs_plane_wave(fda_plan *plan, const double d[3], void *rhs_dev, void *stream)
{
    return guarded([&] {
        if (!plan || !d || !rhs_dev) throw std::invalid_argument("null argument");
        const double n2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (!(n2 > 0)) throw std::invalid_argument("zero direction");
        const double s = 1.0 / std::sqrt(n2);
        const double dd[3] = {d[0] * s, d[1] * s, d[2] * s};
        device_rhs_plane_wave(*plan->P, dd, (double2 *)rhs_dev, (hipStream_t)stream);
        return FDA_OK;
    });
}

int fda_rhs_neumann(fda_plan *plan, const void *q_dev, void *rhs_dev, void *stream)
{
    return guarded([&] {
        if (!plan || !q_dev || !rhs_dev) throw std::invalid_argument("null argument");
        if (q_dev == rhs_dev) throw std::invalid_argument("q and rhs must not alias");
        Plan &P = *plan->P;
        if (!P.has_corr_g)
            throw std::invalid_argument("the Neumann right-hand side needs a plan built with elements and corrections & 2");
        device_rhs_neumann(P, (const double2 *)q_dev, (double2 *)rhs_dev, (hipStream_t)stream);
        return FDA_OK;
    });
}

int fda_stats(const fda_plan *plan, char *buf, size_t len)
{
    return guarded([&] {
        if (!plan || !buf) throw std::invalid_argument("null argument");
        const Plan &P = *plan->P;
        std::string s = plan_stats(P);
        s.pop_back();  // strip the closing brace to append device figures
        s += ", \"device_bytes\": " + std::to_string(P.dev ? P.dev->bytes : 0);
        if (P.dev) {
            int tile = 0, chunk = 0;
            size_t shm = 0;
            for (const auto &T : P.dev->m2lt)
                if (T.n_tiles) tile = T.tile, chunk = T.chunk, shm = std::max(shm, T.shm);
            int maxsh = 0;
            (void)hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, P.dev->device);
            static const char *tune_keys[3] = {"m2l_autotune", "m2m_autotune", "l2l_autotune"};
            for (int kind = 0; kind < 3; ++kind) {
                s += std::string(", \"") + tune_keys[kind] + "\": [";
                bool first = true;
                for (const auto &a : P.dev->autotune) {
                    if ((int)a[4] != kind) continue;
                    char buf[200];
                    std::snprintf(buf, sizeof buf,
                                  "%s{\"level\": %d, \"pairs_per_chunk\": %d, \"ms_16\": %.4f, \"ms_32\": %.4f, "
                                  "\"kernel\": \"%s\"}",
                                  first ? "" : ", ", (int)a[0], (int)a[1], a[2], a[3] < 1e29 ? a[3] : -1.0,
                                  a[5] > 0 ? "wavefront" : "workgroup");
                    s += buf;
                    first = false;
                }
                s += "]";
            }
            s += ", \"graphs_captured\": " + std::to_string(P.dev->graphs.size());
            s += ", \"m2l_mode\": " + std::to_string(P.dev->m2l_mode) + ", \"m2l_tile\": " + std::to_string(tile) +
                 ", \"m2l_chunk\": " + std::to_string(chunk) + ", \"m2l_lds_bytes\": " + std::to_string(shm) +
                 ", \"max_lds_per_block\": " + std::to_string(maxsh) + ", \"m2l_tiles\": [";
            for (size_t l = 0; l < P.dev->tile_stats.size(); ++l) {
                const auto &t = P.dev->tile_stats[l];
                s += (l ? ", [" : "[") + std::to_string(t[0]) + ", " + std::to_string(t[1]) + ", " + std::to_string(t[2]) +
                     ", " + std::to_string(t[3]) + "]";
            }
            s += "]";
        }
        s += ", \"phase_ms\": [";
        for (int t = 0; t < 8; ++t) s += (t ? ", " : "") + std::to_string(P.dev ? P.dev->phase_ms[t] : 0.0);
        s += "]}";
        if (s.size() + 1 > len) throw std::invalid_argument("stats buffer too small");
        std::memcpy(buf, s.c_str(), s.size() + 1);
        return FDA_OK;
    });
}

int fda_set_timing(fda_plan *plan, int on)
{
    return guarded([&] {
        if (!plan) throw std::invalid_argument("null plan");
        plan->P->dev->timing = on ? 1 : 0;
        return FDA_OK;
    });
}

int fda_phase_times(fda_plan *plan, double *ms, int n)
{
    return guarded([&] {
        if (!plan || !ms || n < 0) throw std::invalid_argument("null argument");
        device_phase_average(*plan->P);
        for (int t = 0; t < n && t < 8; ++t) ms[t] = plan->P->dev->phase_ms[t];
        return FDA_OK;
    });
}

int fda_set_graph(fda_plan *plan, int on)
{
    return guarded([&] {
        if (!plan) throw std::invalid_argument("null plan");
        plan->P->dev->use_graph = on ? 1 : 0;
        if (!on) graph_release(*plan->P->dev);
        return FDA_OK;
    });
}

int fda_batch_create(fda_plan *const *plans, int n, fda_batch **out)
{
    return guarded([&] {
        if (!plans || !out || n <= 0) throw std::invalid_argument("bad batch arguments");
        std::vector<Plan *> ps(n);
        for (int i = 0; i < n; ++i) {
            if (!plans[i]) throw std::invalid_argument("null plan in batch");
            ps[i] = plans[i]->P;
            for (int j = 0; j < i; ++j)
                if (ps[j] == ps[i]) throw std::invalid_argument("a plan appears twice in the batch");
        }
        *out = new fda_batch{batch_create(ps.data(), n), std::vector<fda_plan *>(plans, plans + n)};
        return FDA_OK;
    });
}

int fda_batch_matvec(fda_batch *b, int op, const void *const *in_dev, void *const *out_dev, void *stream)
{
    return guarded([&] {
        if (!b || !in_dev || !out_dev) throw std::invalid_argument("null argument");
        for (size_t i = 0; i < b->plans.size(); ++i) {
            const Plan &P = *b->plans[i]->P;
            if (!in_dev[i] || !out_dev[i]) throw std::invalid_argument("null vector in batch");
            if (in_dev[i] == out_dev[i]) throw std::invalid_argument("input and output must not alias");
            check_op(P, op);
        }
        batch_matvec(b->B, op, (const double2 *const *)in_dev, (double2 *const *)out_dev, (hipStream_t)stream);
        return FDA_OK;
    });
}

int fda_batch_solve(fda_batch *b, int op, const void *const *rhs_dev, double tol, int maxit, int restart,
                    int precond, void *const *x_dev, int *iters, double *relres, int *status)
{
    return guarded([&] {
        if (!b || !rhs_dev || !x_dev || !status) throw std::invalid_argument("null argument");
        if (!(tol > 0) || maxit <= 0 || restart <= 0) throw std::invalid_argument("bad GMRES parameters");
        if (precond < 0 || precond > 3) throw std::invalid_argument("unknown preconditioner");
        for (size_t i = 0; i < b->plans.size(); ++i) {
            const Plan &P = *b->plans[i]->P;
            if (!rhs_dev[i] || !x_dev[i]) throw std::invalid_argument("null vector in batch");
            check_op(P, op);
            if (precond && !P.has_corr) throw std::invalid_argument("preconditioner needs elements");
        }
        const int bad = batch_solve(b->B, op, (const double2 *const *)rhs_dev, tol, maxit, restart, precond,
                                    (double2 *const *)x_dev, iters, relres, status);
        return bad ? FDA_NOT_CONVERGED : FDA_OK;
    });
}

void fda_batch_destroy(fda_batch *b)
{
    if (!b) return;
    try {
        batch_destroy(b->B);
    } catch (...) {
    }
    delete b;
}

int fda_net_num_params(void) { return learned_num_params(); }

int fda_net_create(uint64_t seed, fda_net **out)
{
    return guarded([&] {
        if (!out) throw std::invalid_argument("null output pointer");
        *out = new fda_net{learned_create(seed)};
        return FDA_OK;
    });
}

void fda_net_destroy(fda_net *net)
{
    if (!net) return;
    try {
        learned_destroy(net->N);
    } catch (...) {
    }
    delete net;
}

int fda_net_get_params(const fda_net *net, double *params)
{
    return guarded([&] {
        if (!net || !params) throw std::invalid_argument("null argument");
        learned_get_params(net->N, params);
        return FDA_OK;
    });
}

int fda_net_set_params(fda_net *net, const double *params)
{
    return guarded([&] {
        if (!net || !params) throw std::invalid_argument("null argument");
        for (int i = 0; i < learned_num_params(); ++i)
            if (!std::isfinite(params[i])) throw std::invalid_argument("non-finite network parameter");
        learned_set_params(net->N, params);
        return FDA_OK;
    });
}

static void need_bm_plan(fda_plan *plan)
{
    if (!plan) throw std::invalid_argument("null plan");
    if (!plan->P->has_corr) throw std::invalid_argument("the learned preconditioner needs a plan built with elements");
}

int fda_net_loss_grad(fda_net *net, fda_plan *plan, double *loss, double *grad)
{
    return guarded([&] {
        if (!net || !loss) throw std::invalid_argument("null argument");
        need_bm_plan(plan);
        *loss = learned_loss_grad(net->N, *plan->P);
        if (grad) learned_get_grad(net->N, grad);
        return FDA_OK;
    });
}

int fda_net_train_step(fda_net *net, fda_plan *plan, double lr, double *loss)
{
    return guarded([&] {
        if (!net || !(lr > 0)) throw std::invalid_argument("bad argument");
        need_bm_plan(plan);
        const double l = learned_train_step(net->N, *plan->P, lr);
        if (loss) *loss = l;
        return FDA_OK;
    });
}

int fda_net_attach(fda_net *net, fda_plan *plan)
{
    return guarded([&] {
        need_bm_plan(plan);
        if (!net) {
            learned_detach(*plan->P);
            return FDA_OK;
        }
        learned_attach(net->N, *plan->P);
        return FDA_OK;
    });
}

int fda_net_weight_blocks(fda_plan *plan, const void *rhs_dev, int iters)
{
    return guarded([&] {
        if (!plan || (iters > 0 && !rhs_dev)) throw std::invalid_argument("null argument");
        if (iters < 0 || iters > 1000) throw std::invalid_argument("iters must lie in [0, 1000]");
        if (!plan->P->has_corr) throw std::invalid_argument("block weights need a plan built with elements");
        return learned_weight_blocks(*plan->P, (const double2 *)rhs_dev, iters) >= 0 ? FDA_OK : FDA_EHIP;
    });
}

int fda_net_loss_grad_raw(fda_net *net, int n_blocks, const int64_t *pair_off, const int *block_n,
                          const int *block_ne, const int64_t *inv_off, const int64_t *target_off, int64_t n_rows,
                          const double *features, const void *block_inv, const void *targets,
                          const double *block_weight, double *loss, double *grad)
{
    return guarded([&] {
        if (!net || !pair_off || !block_n || !block_ne || !inv_off || !target_off || !features || !block_inv ||
            !targets || !loss)
            throw std::invalid_argument("null argument");
        if (n_blocks <= 0 || n_rows <= 0) throw std::invalid_argument("empty problem");
        *loss = learned_loss_grad_raw(net->N, n_blocks, pair_off, block_n, block_ne, inv_off, target_off, n_rows,
                                      features, (const double2 *)block_inv, (const double2 *)targets, block_weight);
        if (grad) learned_get_grad(net->N, grad);
        return FDA_OK;
    });
}

void fda_destroy(fda_plan *plan)
{
    if (!plan) return;
    try {
        device_free(*plan->P);
    } catch (...) {
    }
    delete plan->P;
    delete plan;
}

const char *fda_last_error(void) { return g_err.c_str(); }

}  // extern "C"
