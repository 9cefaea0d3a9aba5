// Host-side plan construction: copies the caller's geometry, sorts it into
// octree order and runs the FP64 set-up stages.
#include <chrono>
#include <cstdio>
#include <cmath>
#include <sstream>
#include <stdexcept>

#include <unordered_map>

#include "plan.hpp"

namespace fdbem {

static double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

Plan *plan_create_host(int64_t n, const double *pts, const double *nrm, const double *w, int64_t n_elem,
                       const double *elem, double k, double eps, const Options &opt)
{
    if (n <= 0 || !pts || !nrm || !w) throw std::invalid_argument("empty geometry");
    if (!(k > 0) || !std::isfinite(k)) throw std::invalid_argument("wavenumber must be positive");
    if (!(eps > 0 && eps < 1)) throw std::invalid_argument("eps must lie in (0,1)");
    if (n_elem > 0 && (n_elem * 6 != n || !elem)) throw std::invalid_argument("elements must carry 6 nodes each");
    if (opt.leaf_cap < 1) throw std::invalid_argument("leaf_cap must be >= 1");
    Plan *P = new Plan();
    try {
        P->N = n;
        P->k = k;
        P->eps = eps;
        P->lambda = 2.0 * M_PI / k;
        P->opt = opt;
        P->px.resize(n);
        P->py.resize(n);
        P->pz.resize(n);
        P->pnx.resize(n);
        P->pny.resize(n);
        P->pnz.resize(n);
        P->pw.resize(n);
        for (int64_t i = 0; i < n; ++i) {
            P->px[i] = pts[3 * i];
            P->py[i] = pts[3 * i + 1];
            P->pz[i] = pts[3 * i + 2];
            P->pnx[i] = nrm[3 * i];
            P->pny[i] = nrm[3 * i + 1];
            P->pnz[i] = nrm[3 * i + 2];
            P->pw[i] = w[i];
            if (!std::isfinite(P->px[i] + P->py[i] + P->pz[i] + P->pw[i]))
                throw std::invalid_argument("non-finite geometry");
        }
        if (n_elem > 0) {
            P->n_elem = n_elem;
            P->elem.assign(elem, elem + 18 * n_elem);
        }
        auto log = [&](const char *what, double t) {
            if (P->opt.verbose) {
                std::fprintf(stderr, "[fdbem] %s %.2f s\n", what, t);
                std::fflush(stderr);
            }
        };
        double t0 = now_s();
        build_tree(*P);
        log("octree", now_s() - t0);
        build_lists(*P);
        double t1 = now_s();
        P->t_setup_tree = t1 - t0;
        log("lists", P->t_setup_tree);
        if (P->opt.far_field) {
            build_templates(*P);
            double t2 = now_s();
            P->t_setup_tmpl = t2 - t1;
            log("templates", P->t_setup_tmpl);
            build_operators(*P);
            P->t_setup_ops = now_s() - t2;
            log("translation operators", P->t_setup_ops);
        }
    } catch (...) {
        delete P;
        throw;
    }
    return P;
}

std::string plan_stats(const Plan &P)
{
    std::ostringstream o;
    o.precision(6);
    o << "{\"N\": " << P.N << ", \"k\": " << P.k << ", \"eps\": " << P.eps << ", \"lambda\": " << P.lambda
      << ", \"root_w\": " << P.root_w << ", \"n_levels\": " << P.levels.size() << ", \"n_leaves\": " << P.leaves.size()
      << ", \"p2p_pairs\": " << P.p2p_pairs << ", \"matpool_bytes\": " << P.matpool.size() * 16
      << ", \"density_slots_out\": " << P.out_total << ", \"density_slots_in\": " << P.in_total
      << ", \"corr_nnz\": " << 6 * P.corr_blocks << ", \"setup_s\": {\"tree\": " << P.t_setup_tree
      << ", \"templates\": " << P.t_setup_tmpl << ", \"operators\": " << P.t_setup_ops
      << ", \"corrections\": " << P.t_setup_corr << "}, \"levels\": [";
    for (size_t l = 0; l < P.levels.size(); ++l) {
        const LevelInfo &L = P.levels[l];
        int64_t npairs = l < P.m2l.size() ? (int64_t)P.m2l[l].size() : 0;
        int nlr = 0, nk = l < P.m2l_nkeys.size() ? P.m2l_nkeys[l] : 0;
        double flops = 0, opbytes = 0;
        if (l < P.m2l_lists.size()) {
            const GemvList &G = P.m2l_lists[l];
            std::unordered_map<int64_t, int> seen;
            for (size_t q = 0; q < G.rank.size(); ++q) {
                const int r = G.rank[q];
                nlr += r >= 0;
                flops += r >= 0 ? 8.0 * r * (G.rows + G.cols) : 8.0 * G.rows * G.cols;
                if (seen.emplace(G.mat_off[q], r).second)
                    opbytes += 16.0 * (r >= 0 ? (double)r * (G.rows + G.cols) : (double)G.rows * G.cols);
            }
        }
        // M2M (child slots of level l+1 -> parent slots of level l) and L2L
        // (parent slots of level l-1 -> child slots of level l): flops of the
        // dense compressed operators, and the minimum bytes: each unique
        // operator, each input slot and each output slot once
        auto list_work = [](const GemvList &G, double &fl, double &by, int64_t &ent) {
            std::unordered_map<int64_t, int> ops;
            std::unordered_map<int64_t, int> ins;
            fl = 0;
            by = 0;
            ent = (int64_t)G.in_off.size();
            for (size_t q = 0; q < G.in_off.size(); ++q) {
                const int r = G.rank[q];
                fl += r >= 0 ? 8.0 * r * (G.rows + G.cols) : 8.0 * G.rows * G.cols;
                if (ops.emplace(G.mat_off[q], 1).second)
                    by += 16.0 * (r >= 0 ? (double)r * (G.rows + G.cols) : (double)G.rows * G.cols);
                if (ins.emplace(G.in_off[q], 1).second) by += 16.0 * G.cols;
            }
            by += 16.0 * G.rows * (double)G.out_off.size();
        };
        double m2m_fl = 0, m2m_by = 0, l2l_fl = 0, l2l_by = 0, m2l_min = 0;
        int64_t m2m_e = 0, l2l_e = 0;
        if (l < P.m2m_lists.size()) list_work(P.m2m_lists[l], m2m_fl, m2m_by, m2m_e);
        if (l < P.l2l_lists.size()) list_work(P.l2l_lists[l], l2l_fl, l2l_by, l2l_e);
        if (l < P.m2l_lists.size()) {
            double fl;
            int64_t e;
            list_work(P.m2l_lists[l], fl, m2l_min, e);
        }
        o << (l ? ", " : "") << "{\"w\": " << L.w << ", \"hf\": " << (L.hf ? 1 : 0) << ", \"m\": " << L.m
          << ", \"cubes\": " << L.cubes.size() << ", \"out_slots\": " << L.n_out << ", \"in_slots\": " << L.n_in
          << ", \"s\": " << (l < P.tmpl.size() ? P.tmpl[l].s : 0)
          << ", \"n_equiv\": " << (l < P.tmpl.size() ? P.tmpl[l].X.size() / 3 : 0)
          << ", \"n_check\": " << (l < P.tmpl.size() ? P.tmpl[l].Y.size() / 3 : 0) << ", \"m2l_pairs\": " << npairs
          << ", \"m2l_ops\": " << nk << ", \"m2l_pairs_lowrank\": " << nlr << ", \"m2l_flops\": " << flops
          << ", \"m2l_op_bytes\": " << opbytes << ", \"m2l_min_bytes\": " << m2l_min
          << ", \"m2m_entries\": " << m2m_e << ", \"m2m_flops\": " << m2m_fl << ", \"m2m_min_bytes\": " << m2m_by
          << ", \"l2l_entries\": " << l2l_e << ", \"l2l_flops\": " << l2l_fl << ", \"l2l_min_bytes\": " << l2l_by
          << "}";
    }
    o << "]";
    // S2M and L2T: kernel evaluations between leaf points and the level's
    // check points, and the complex multiply-adds of W (s x |Y|) per leaf
    auto leaf_work = [&](const std::vector<LeafTask> &T, double &ev, double &wf) {
        ev = 0;
        wf = 0;
        for (const LeafTask &t : T) {
            const LevelTemplate &L = P.tmpl[t.tmpl];
            const double ny = (double)(L.Y.size() / 3);
            ev += (double)(t.end - t.start) * ny;
            wf += 8.0 * L.s * ny;
        }
    };
    double s2m_ev, s2m_wf, l2t_ev, l2t_wf;
    leaf_work(P.s2m_tasks, s2m_ev, s2m_wf);
    leaf_work(P.l2t_tasks, l2t_ev, l2t_wf);
    o << ", \"s2m_evals\": " << s2m_ev << ", \"s2m_w_flops\": " << s2m_wf << ", \"l2t_evals\": " << l2t_ev
      << ", \"l2t_w_flops\": " << l2t_wf << ", \"n_s2m_tasks\": " << P.s2m_tasks.size()
      << ", \"n_l2t_tasks\": " << P.l2t_tasks.size() << "}";
    return o.str();
}

}  // namespace fdbem
