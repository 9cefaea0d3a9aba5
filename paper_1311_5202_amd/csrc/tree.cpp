// Adaptive octree, near/interaction lists and directional wedges of the fast
// directional algorithm (paper section 3.1.1).
//
// * Root: a cube of width lambda * 2^M (smallest such width covering the
//   points), so that every level is either low frequency (w < lambda) or high
//   frequency with an integer number m = w / lambda of wedge cells per face
//   edge.  Cubes with more than leaf_cap points are split; with leaf_rule 0
//   every high-frequency cube holding points is split as well, so leaves are
//   low-frequency cubes.
// * Near field of same-level cubes B, C: low frequency -> adjacent (gap <= 0);
//   high frequency -> gap <= c_d k w^2 with gap = max_i |c_B,i - c_C,i| - w.
// * Lists by a dual traversal from (root, root): a near pair of non-leaf
//   cubes passes its child pairs on; child pairs that are not near form the
//   interaction field I = N^P \ N^C (an M2L); a near pair with a leaf is
//   summed directly (P2P) between the two subtrees.  Every point pair is
//   covered exactly once.
// * A far pair whose point counts multiply to at most p2p_threshold is summed
//   directly instead (its translation would cost more than the point pairs).
// * Wedges: each cube face is cut into an m x m grid of cells; a direction
//   belongs to the cell its central projection hits.  Cells of a parent level
//   (2m) nest in cells of the child level (m).
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <unordered_map>

#include "plan.hpp"

namespace fdbem {

// ------------------------------------------------------------------ wedges
int wedge_of(const double v[3], int m)
{
    int ax = 0;
    double best = std::fabs(v[0]);
    for (int d = 1; d < 3; ++d)
        if (std::fabs(v[d]) > best) {
            best = std::fabs(v[d]);
            ax = d;
        }
    const int f = 2 * ax + (v[ax] < 0 ? 1 : 0);
    const int j = (ax + 1) % 3, l = (ax + 2) % 3;
    const double u = v[j] / best, t = v[l] / best;
    int iu = (int)std::floor((u + 1.0) * 0.5 * m);
    int it = (int)std::floor((t + 1.0) * 0.5 * m);
    iu = std::min(std::max(iu, 0), m - 1);
    it = std::min(std::max(it, 0), m - 1);
    return f * m * m + iu * m + it;
}

int wedge_neg(int z, int m)
{
    const int f = z / (m * m), rem = z % (m * m);
    const int iu = rem / m, it = rem % m;
    return (f ^ 1) * m * m + (m - 1 - iu) * m + (m - 1 - it);
}

int wedge_child(int z, int m)
{
    const int f = z / (m * m), rem = z % (m * m);
    const int iu = rem / m, it = rem % m;
    const int mc = m / 2;
    return f * mc * mc + (iu / 2) * mc + (it / 2);
}

void wedge_center(int z, int m, double c[3])
{
    const int f = z / (m * m), rem = z % (m * m);
    const int iu = rem / m, it = rem % m;
    const int ax = f / 2;
    const double sg = (f & 1) ? -1.0 : 1.0;
    const int j = (ax + 1) % 3, l = (ax + 2) % 3;
    c[ax] = sg;
    c[j] = (2.0 * iu + 1.0 - m) / m;
    c[l] = (2.0 * it + 1.0 - m) / m;
}

static std::array<double, 9> rotation_from_x(const double dir[3])
{
    // Rodrigues rotation taking e_x to the unit vector dir
    const double c = dir[0];
    std::array<double, 9> R{};
    const double ax[3] = {0.0, -dir[2], dir[1]};  // e_x x dir
    const double s = std::sqrt(ax[1] * ax[1] + ax[2] * ax[2]);
    if (s < 1e-14) {
        R = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        if (c < 0) R = {-1, 0, 0, 0, -1, 0, 0, 0, 1};
        return R;
    }
    const double k[3] = {ax[0] / s, ax[1] / s, ax[2] / s};
    const double K[9] = {0, -k[2], k[1], k[2], 0, -k[0], -k[1], k[0], 0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double t = 0;
            for (int l = 0; l < 3; ++l) t += K[3 * i + l] * K[3 * l + j];
            K2[3 * i + j] = t;
        }
    for (int i = 0; i < 9; ++i) R[i] = ((i % 4) == 0 ? 1.0 : 0.0) + s * K[i] + (1.0 - c) * K2[i];
    return R;
}

WedgeFrame wedge_frame(int z, int m)
{
    double c[3];
    wedge_center(z, m, c);
    std::array<int, 3> perm = {0, 1, 2};
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return std::fabs(c[a]) > std::fabs(c[b]); });
    WedgeFrame F;
    F.perm = perm;
    const int s0 = c[perm[0]] < 0 ? -1 : 1;
    double c0[3];
    for (int i = 0; i < 3; ++i) {
        const double v = c[perm[i]];
        F.sign[i] = (v == 0.0) ? s0 : (v < 0 ? -1 : 1);
        c0[i] = std::fabs(v);
    }
    F.orbit = wedge_of(c0, m);
    const double nrm = std::sqrt(c0[0] * c0[0] + c0[1] * c0[1] + c0[2] * c0[2]);
    const double d0[3] = {c0[0] / nrm, c0[1] / nrm, c0[2] / nrm};
    const std::array<double, 9> R0 = rotation_from_x(d0);
    // g as a matrix: column i is sign[i] e_perm[i]
    double g[9] = {0};
    for (int i = 0; i < 3; ++i) g[3 * perm[i] + i] = F.sign[i];
    for (int i = 0; i < 9; ++i) F.G[i] = g[i];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double t = 0;
            for (int l = 0; l < 3; ++l) t += g[3 * i + l] * R0[3 * l + j];
            F.R[3 * i + j] = t;
        }
    return F;
}

// ------------------------------------------------------------------ tree
void build_tree(Plan &P)
{
    const int64_t N = P.N;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < N; ++i) {
        const double p[3] = {P.px[i], P.py[i], P.pz[i]};
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], p[d]);
            hi[d] = std::max(hi[d], p[d]);
        }
    }
    double D = 0;
    for (int d = 0; d < 3; ++d) {
        P.root_center[d] = 0.5 * (lo[d] + hi[d]);
        D = std::max(D, hi[d] - lo[d]);
    }
    D = std::max(D, 1e-12) * (1.0 + 1e-9);
    const int M = (int)std::ceil(std::log2(D / P.lambda));
    P.root_w = P.lambda * std::ldexp(1.0, M);
    if (P.root_w < D) P.root_w *= 2;

    std::vector<int64_t> idx(N), tmp(N);
    for (int64_t i = 0; i < N; ++i) idx[i] = i;
    P.cubes.clear();
    P.cubes.emplace_back();
    Cube &root = P.cubes[0];
    root.level = 0;
    root.start = 0;
    root.end = N;
    root.ijk[0] = root.ijk[1] = root.ijk[2] = 0;
    std::vector<int> frontier = {0};
    int level = 0;
    const double corner[3] = {P.root_center[0] - 0.5 * P.root_w, P.root_center[1] - 0.5 * P.root_w,
                              P.root_center[2] - 0.5 * P.root_w};
    while (!frontier.empty()) {
        const double w = P.root_w * std::ldexp(1.0, -level);
        const bool hf = w >= P.lambda * (1.0 - 1e-9);
        std::vector<int> next;
        for (int cid : frontier) {
            const int64_t s = P.cubes[cid].start, e = P.cubes[cid].end, cnt = e - s;
            bool split = cnt > P.opt.leaf_cap || (P.opt.leaf_rule == 0 && hf && cnt > 0);
            if (!P.opt.far_field) split = false;
            if (level >= 40) split = false;
            if (!split) continue;
            const double cx = corner[0] + (P.cubes[cid].ijk[0] + 0.5) * w;
            const double cy = corner[1] + (P.cubes[cid].ijk[1] + 0.5) * w;
            const double cz = corner[2] + (P.cubes[cid].ijk[2] + 0.5) * w;
            int64_t count[8] = {0};
            std::vector<unsigned char> oct(cnt);
            for (int64_t t = 0; t < cnt; ++t) {
                const int64_t i = idx[s + t];
                const int o = (P.px[i] >= cx ? 1 : 0) | (P.py[i] >= cy ? 2 : 0) | (P.pz[i] >= cz ? 4 : 0);
                oct[t] = (unsigned char)o;
                count[o]++;
            }
            int64_t off[8];
            off[0] = s;
            for (int o = 1; o < 8; ++o) off[o] = off[o - 1] + count[o - 1];
            int64_t pos[8];
            std::memcpy(pos, off, sizeof(pos));
            for (int64_t t = 0; t < cnt; ++t) tmp[pos[oct[t]]++] = idx[s + t];
            std::memcpy(idx.data() + s, tmp.data() + s, sizeof(int64_t) * cnt);
            P.cubes[cid].leaf = false;
            for (int o = 0; o < 8; ++o) {
                if (count[o] == 0) continue;
                Cube c;
                c.level = level + 1;
                c.start = off[o];
                c.end = off[o] + count[o];
                c.parent = cid;
                c.ijk[0] = 2 * P.cubes[cid].ijk[0] + (o & 1);
                c.ijk[1] = 2 * P.cubes[cid].ijk[1] + ((o >> 1) & 1);
                c.ijk[2] = 2 * P.cubes[cid].ijk[2] + ((o >> 2) & 1);
                const int nid = (int)P.cubes.size();
                P.cubes.push_back(c);
                P.cubes[cid].child[o] = nid;
                next.push_back(nid);
            }
        }
        frontier.swap(next);
        ++level;
    }
    // permute point arrays into tree order
    P.perm = idx;
    auto permute = [&](std::vector<double> &a) {
        std::vector<double> b(N);
        for (int64_t i = 0; i < N; ++i) b[i] = a[idx[i]];
        a.swap(b);
    };
    permute(P.px);
    permute(P.py);
    permute(P.pz);
    permute(P.pnx);
    permute(P.pny);
    permute(P.pnz);
    permute(P.pw);
    // levels
    int nlev = 0;
    for (const Cube &c : P.cubes) nlev = std::max(nlev, c.level + 1);
    P.levels.assign(nlev, LevelInfo());
    for (int l = 0; l < nlev; ++l) {
        LevelInfo &L = P.levels[l];
        L.level = l;
        L.w = P.root_w * std::ldexp(1.0, -l);
        L.hf = L.w >= P.lambda * (1.0 - 1e-9);
        L.m = L.hf ? P.opt.wedge_factor * (int)std::lround(L.w / P.lambda) : 0;
        L.nwedge = L.hf ? 6 * L.m * L.m : 1;
    }
    P.leaves.clear();
    for (int id = 0; id < (int)P.cubes.size(); ++id) {
        Cube &c = P.cubes[id];
        c.local = (int)P.levels[c.level].cubes.size();
        P.levels[c.level].cubes.push_back(id);
        if (c.leaf) P.leaves.push_back(id);
    }
}

static inline int cheb(const Cube &a, const Cube &b)
{
    int d = 0;
    for (int t = 0; t < 3; ++t) d = std::max(d, std::abs(a.ijk[t] - b.ijk[t]));
    return d;
}

// maximal Chebyshev offset (in cube widths) that is still near at a level
static int near_reach(const Plan &P, const LevelInfo &L)
{
    if (!L.hf) return 1;
    return (int)std::floor(P.opt.c_d * P.k * L.w + 1e-9) + 1;
}

static void subtree_leaves(const Plan &P, int cid, std::vector<int> &out)
{
    const Cube &c = P.cubes[cid];
    if (c.leaf) {
        out.push_back(cid);
        return;
    }
    for (int o = 0; o < 8; ++o)
        if (c.child[o] >= 0) subtree_leaves(P, c.child[o], out);
}

void build_lists(Plan &P)
{
    const int nlev = (int)P.levels.size();
    P.m2l.assign(nlev, {});
    std::vector<std::vector<std::pair<int, int>>> m2l_raw(nlev);
    std::vector<std::pair<int, int>> p2p_raw;
    std::vector<std::pair<int, int>> nearp = {{0, 0}};
    for (int l = 0; l < nlev && !nearp.empty(); ++l) {
        std::vector<std::pair<int, int>> next;
        const int reach_c = (l + 1 < nlev) ? near_reach(P, P.levels[l + 1]) : 1;
        for (auto [b, c] : nearp) {
            const Cube &B = P.cubes[b], &C = P.cubes[c];
            if (B.leaf || C.leaf) {
                p2p_raw.push_back({b, c});
                continue;
            }
            for (int ob = 0; ob < 8; ++ob) {
                const int cb = B.child[ob];
                if (cb < 0) continue;
                for (int oc = 0; oc < 8; ++oc) {
                    const int cc = C.child[oc];
                    if (cc < 0) continue;
                    if (cheb(P.cubes[cb], P.cubes[cc]) <= reach_c)
                        next.push_back({cb, cc});
                    else if ((double)(P.cubes[cb].end - P.cubes[cb].start) * (double)(P.cubes[cc].end - P.cubes[cc].start) <=
                             P.opt.p2p_threshold)
                        p2p_raw.push_back({cb, cc});  // cheaper summed directly than translated
                    else
                        m2l_raw[l + 1].push_back({cb, cc});
                }
            }
        }
        nearp.swap(next);
    }
    // ---- P2P: per target leaf, the source ranges
    const int nleaf = (int)P.leaves.size();
    std::vector<int> leaf_index(P.cubes.size(), -1);
    for (int t = 0; t < nleaf; ++t) leaf_index[P.leaves[t]] = t;
    std::vector<std::vector<std::pair<int64_t, int64_t>>> src(nleaf);
    std::vector<int> tl;
    for (auto [b, c] : p2p_raw) {
        tl.clear();
        subtree_leaves(P, b, tl);
        for (int t : tl) src[leaf_index[t]].push_back({P.cubes[c].start, P.cubes[c].end});
    }
    P.p2p_tgt_start.resize(nleaf);
    P.p2p_tgt_end.resize(nleaf);
    P.p2p_ptr.assign(nleaf + 1, 0);
    P.p2p_src_start.clear();
    P.p2p_src_end.clear();
    P.p2p_pairs = 0;
    for (int t = 0; t < nleaf; ++t) {
        const Cube &L = P.cubes[P.leaves[t]];
        P.p2p_tgt_start[t] = L.start;
        P.p2p_tgt_end[t] = L.end;
        auto &v = src[t];
        std::sort(v.begin(), v.end());
        std::vector<std::pair<int64_t, int64_t>> merged;
        for (auto r : v) {
            if (!merged.empty() && merged.back().second == r.first)
                merged.back().second = r.second;
            else
                merged.push_back(r);
        }
        for (auto r : merged) {
            P.p2p_src_start.push_back(r.first);
            P.p2p_src_end.push_back(r.second);
            P.p2p_pairs += (r.second - r.first) * (L.end - L.start);
        }
        P.p2p_ptr[t + 1] = (int)P.p2p_src_start.size();
    }
    // ---- M2L: wedges, slots, operator keys
    P.m2l_nkeys.assign(nlev, 0);
    P.m2l_keyinfo.assign(nlev, {});
    std::vector<std::vector<int>> pair_zeta(nlev);
    std::vector<std::vector<int>> key_of(nlev);
    for (int l = 0; l < nlev; ++l) {
        LevelInfo &L = P.levels[l];
        const size_t np = m2l_raw[l].size();
        pair_zeta[l].resize(np);
        key_of[l].resize(np);
        std::unordered_map<int64_t, int> keymap;
        if (L.hf) {
            L.frames.resize(L.nwedge);
            for (int z = 0; z < L.nwedge; ++z) L.frames[z] = wedge_frame(z, L.m);
        }
        for (size_t q = 0; q < np; ++q) {
            const Cube &B = P.cubes[m2l_raw[l][q].first], &C = P.cubes[m2l_raw[l][q].second];
            int d[3] = {B.ijk[0] - C.ijk[0], B.ijk[1] - C.ijk[1], B.ijk[2] - C.ijk[2]};
            int64_t code;
            if (L.hf) {
                const double v[3] = {(double)d[0], (double)d[1], (double)d[2]};
                const int z = wedge_of(v, L.m);
                pair_zeta[l][q] = z;
                const WedgeFrame &F = L.frames[z];
                int del[3];
                for (int i = 0; i < 3; ++i) del[i] = F.sign[i] * d[F.perm[i]];
                code = (((int64_t)F.orbit * 4096 + (del[0] + 2048)) * 4096 + (del[1] + 2048)) * 4096 + (del[2] + 2048);
            } else {
                pair_zeta[l][q] = 0;
                code = ((int64_t)(d[0] + 2048) * 4096 + (d[1] + 2048)) * 4096 + (d[2] + 2048);
            }
            auto it = keymap.find(code);
            int key;
            if (it == keymap.end()) {
                key = (int)keymap.size();
                keymap.emplace(code, key);
                if (L.hf) {
                    const WedgeFrame &F = L.frames[pair_zeta[l][q]];
                    std::array<int, 4> ki;
                    ki[0] = F.orbit;
                    for (int i = 0; i < 3; ++i) ki[1 + i] = F.sign[i] * d[F.perm[i]];
                    P.m2l_keyinfo[l].push_back(ki);
                } else {
                    P.m2l_keyinfo[l].push_back({-1, d[0], d[1], d[2]});
                }
            } else
                key = it->second;
            key_of[l][q] = key;
        }
        P.m2l_nkeys[l] = (int)keymap.size();
    }
    // slot marking, top-down
    for (int l = 0; l < nlev; ++l) {
        LevelInfo &L = P.levels[l];
        const size_t nc = L.cubes.size();
        L.out_slot.assign(nc * L.nwedge, -1);
        L.in_slot.assign(nc * L.nwedge, -1);
        std::vector<char> need_out(nc * L.nwedge, 0), need_in(nc * L.nwedge, 0);
        for (size_t q = 0; q < m2l_raw[l].size(); ++q) {
            const Cube &B = P.cubes[m2l_raw[l][q].first], &C = P.cubes[m2l_raw[l][q].second];
            const int z = pair_zeta[l][q];
            const int zn = L.hf ? wedge_neg(z, L.m) : 0;
            need_out[(size_t)C.local * L.nwedge + z] = 1;
            need_in[(size_t)B.local * L.nwedge + zn] = 1;
        }
        if (l > 0) {
            const LevelInfo &Pp = P.levels[l - 1];
            for (size_t a = 0; a < Pp.cubes.size(); ++a) {
                const Cube &Par = P.cubes[Pp.cubes[a]];
                for (int zp = 0; zp < Pp.nwedge; ++zp) {
                    const bool po = Pp.out_slot[a * Pp.nwedge + zp] >= 0;
                    const bool pi = Pp.in_slot[a * Pp.nwedge + zp] >= 0;
                    if (!po && !pi) continue;
                    const int zc = L.hf ? wedge_child(zp, Pp.m) : 0;
                    for (int o = 0; o < 8; ++o) {
                        if (Par.child[o] < 0) continue;
                        const Cube &Ch = P.cubes[Par.child[o]];
                        if (po) need_out[(size_t)Ch.local * L.nwedge + zc] = 1;
                        if (pi) need_in[(size_t)Ch.local * L.nwedge + zc] = 1;
                    }
                }
            }
        }
        int no = 0, ni = 0;
        for (size_t t = 0; t < need_out.size(); ++t) {
            if (need_out[t]) L.out_slot[t] = no++;
            if (need_in[t]) L.in_slot[t] = ni++;
        }
        L.n_out = no;
        L.n_in = ni;
        // pairs in slot form
        auto &V = P.m2l[l];
        V.resize(m2l_raw[l].size());
        for (size_t q = 0; q < m2l_raw[l].size(); ++q) {
            const Cube &B = P.cubes[m2l_raw[l][q].first], &C = P.cubes[m2l_raw[l][q].second];
            const int z = pair_zeta[l][q];
            const int zn = L.hf ? wedge_neg(z, L.m) : 0;
            V[q].src_slot = L.out_slot[(size_t)C.local * L.nwedge + z];
            V[q].tgt_slot = L.in_slot[(size_t)B.local * L.nwedge + zn];
            V[q].key = key_of[l][q];
        }
        std::sort(V.begin(), V.end(), [](const M2LPair &a, const M2LPair &b) {
            return a.tgt_slot != b.tgt_slot ? a.tgt_slot < b.tgt_slot : a.key < b.key;
        });
    }
}

}  // namespace fdbem
