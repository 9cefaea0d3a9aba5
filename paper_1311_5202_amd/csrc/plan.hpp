// Internal plan of the fast directional Burton-Miller mat-vec: the host-side
// set-up (octree, interaction lists, directional wedges, point templates and
// compressed translation operators) and the device-resident copy the HIP
// kernels read.  Not part of the public C ABI.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "hostkernels.hpp"
#include "linalg.hpp"

namespace fdbem {

struct Options {
    double svd_eps = 0;      // truncation of the pseudo-inverses (0 -> eps)
    double lowrank_eps = 0;  // truncation of the M2L low-rank factors (0 -> eps)
    int leaf_cap = 64;       // max points per leaf
    int leaf_rule = 0;       // 0: leaves are low-frequency cubes (w < lambda)
    int wedge_factor = 2;    // wedge cells per face edge = wedge_factor * w / lambda
    int m2l_tile = 0;        // M2L target tile (0 auto, <0 per-target GEMV kernel)
    double p2p_threshold = 400;   // far pairs with n_B * n_C <= this are summed directly
    double c_d = 1.0 / M_PI; // high-frequency near-field constant
    int far_field = 1;       // 0: every pair by direct summation (debug / tiny problems)
    int lf_grid = 0;         // points per edge of the low-frequency surface grids (0 -> auto)
    int precision = 0;       // 0 FP64, 1 FP32 far field
    int corrections = 1;     // build local corrections when elements are supplied
    int verbose = 0;
    double coupling = 1.0;   // Burton-Miller alpha = i coupling / k
    int hf_template = 0;     // 0: checks on the region each wedge's field is evaluated in, cube-surface
                             // equivalents; 1: circular check cone, ball equivalents (earlier construction)
    int original = 0;        // 1: translations on equivalent densities with uncompressed R+ and K, no
                             // low-rank M2L (the paper's comparison method, Table 1)
    int autotune = 1;        // time the M2L/M2M/L2L chunk shapes on the plan and keep the faster
    int slab_mb = 1024;      // scratch of per-pair translation results per slab (MiB)
    int serial_slabs = 0;    // 0: two slab buffers, each launch also sums the previous slab; 1: one buffer
    int chunk_kernel = 0;    // 0: wavefront chunk kernel where an operator fits it; 1: workgroup kernel only
    // k of the coupling: alpha = i / alpha_k()
    double alpha_k(double k) const { return k / coupling; }
};

struct Cube {
    int level = 0;
    int64_t start = 0, end = 0;  // range in sorted point order (whole subtree)
    int parent = -1;
    int child[8];
    int ijk[3];
    int local = 0;               // index within its level
    bool leaf = true;
    Cube() { for (int &c : child) c = -1; }
};

// Equivalent and check points of one high-frequency wedge orbit, in the
// frame of the orbit's representative wedge (relative to the cube centre),
// with their reduced bases (eqs. eq_svdr, eq_invr).
struct OrbitTemplate {
    std::vector<double> X;  // equivalent points, |X| x 3
    std::vector<double> Y;  // check points, |Y| x 3
    CMat Vt;                // |X| x s, zero columns past this orbit's own rank
    CMat W;                 // s x |Y|, zero rows past this orbit's own rank
    std::vector<double> sing;
    int rank = 0;           // singular values kept for this orbit (<= s of the level)
};

// Point templates and pseudo-inverse of one level (section 3.1.2 and eqs.
// eq_svdr, eq_invr).  Low-frequency templates are axis-aligned cube
// surfaces (X, Y, Vt, W below).  High-frequency levels hold one template per
// wedge orbit of the 48 signed permutations of the cube (`orbit`); the
// template of wedge z is that of its orbit mapped by the signed permutation
// of its frame, which maps the cube onto itself.
struct LevelTemplate {
    bool hf = false;
    double w = 0;
    int m = 0;            // wedges per face edge (high frequency), 0 for low frequency
    int s = 0;            // reduced dimension
    std::vector<double> X;  // equivalent points, |X| x 3, relative to the cube centre
    std::vector<double> Y;  // check points, |Y| x 3, relative to the cube centre
    CMat Vt;              // |X| x s  (V~)
    CMat W;               // s x |Y|  (Sigma~^-1 U~^H)
    std::vector<double> sing;  // singular values of R
    double theta_cone = 0, r_in = 0, r_out = 0;
    std::unordered_map<int, OrbitTemplate> orbit;  // high frequency: by representative wedge
    int n_equiv_max = 0, n_check_max = 0;
};

struct WedgeFrame {
    std::array<double, 9> R;   // rotation (row-major) taking the +x direction to this wedge
    std::array<double, 9> G;   // signed permutation (row-major) taking the orbit's representative to this wedge
    int orbit = 0;             // canonical wedge id of its symmetry orbit
    std::array<int, 3> perm;   // signed permutation g: g e_i = sign[i] e_perm[i]
    std::array<int, 3> sign;
};

struct LevelInfo {
    int level = 0;
    double w = 0;
    bool hf = false;
    int m = 0;
    int nwedge = 1;
    std::vector<int> cubes;         // cube ids at this level
    std::vector<int> out_slot;      // (local cube * nwedge + wedge) -> slot, -1 if unused
    std::vector<int> in_slot;
    int n_out = 0, n_in = 0;
    int64_t out_base = 0, in_base = 0;  // offsets (complex elements) in the density arrays
    std::vector<WedgeFrame> frames;     // per wedge (high frequency)
};

struct M2LPair {
    int tgt_slot, src_slot;  // level-local slots
    int key;                 // level-local unique operator id
};

// A batched GEMV task list: out[o] += sum_e op(Mat_e) in[e].
struct GemvList {
    std::vector<int64_t> out_off;    // per output slot: offset (complex elements)
    std::vector<int> ptr;            // CSR over output slots (size n_out+1)
    std::vector<int64_t> in_off;     // per entry
    std::vector<int64_t> mat_off;    // per entry: offset into the matrix pool (complex elements)
    std::vector<int> rank;           // per entry: -1 dense, else low-rank r (U then V stored)
    int rows = 0, cols = 0;          // output / input dimension
    int trans = 0;                   // 1: use Mat^T (L2L)
    std::vector<int> out_wedge;      // per output slot: its wedge (M2L tiling order)
};

// M2L in target tiles: every tile owns up to `tile` target slots of one level
// (same wedge, consecutive cubes in octree order); its pairs are grouped into chunks that share one operator and hit
// distinct targets, so a workgroup reuses each operator across the chunk and
// accumulates its targets in LDS without atomics.
struct M2LTiles {
    int tile = 0, chunk = 0, s = 0, max_rank = 0;
    std::vector<int64_t> tgt_off;    // per target slot (tile q owns entries q*tile ..): density offset
    std::vector<int> tile_ntgt;      // per tile: number of target slots
    std::vector<int> tile_cptr;      // per tile: chunk range (size n_tiles+1)
    std::vector<int64_t> ch_mat;     // per chunk: operator offset in the pool
    std::vector<int> ch_rank;        // per chunk: -1 dense, else low-rank r
    std::vector<int> ch_pptr;        // per chunk: pair range (size n_chunks+1)
    std::vector<int> pr_tl;          // per pair: target index within the tile
    std::vector<int64_t> pr_src;     // per pair: source density offset
};

// M2L by operator: pairs sharing one compressed operator are cut into chunks
// of at most `chunk` pairs; one wavefront applies the operator to a chunk and
// adds the results to the targets with FP64 atomics.
struct M2LChunks {
    int chunk = 0, s = 0, cols = 0, max_rank = 0, trans = 0;
    std::vector<int64_t> ch_mat;
    std::vector<int> ch_rank, ch_pptr;
    std::vector<int64_t> pr_tgt, pr_src;
    std::vector<int64_t> pr_pos;     // per pair: entry index in the slab (target-major)
    std::vector<int64_t> red_out;    // per output of the slab: offset
    std::vector<int64_t> red_ptr;    // per output of the slab: entry range (size n_out+1)
};

struct LeafTask {
    int64_t start, end;     // sorted point range
    int64_t slot_off;       // density offset (complex elements)
    int tmpl;               // level id of the template
    double center[3];       // cube centre
};

struct Plan {
    // problem
    int64_t N = 0;
    double k = 0, eps = 0, lambda = 0;
    Options opt;
    // points in sorted (tree) order
    std::vector<double> px, py, pz, pnx, pny, pnz, pw;
    std::vector<int64_t> perm;      // sorted index -> caller index
    // elements (for local corrections)
    int64_t n_elem = 0;
    std::vector<double> elem;       // n_elem * 18
    // tree
    double root_center[3] = {0, 0, 0};
    double root_w = 0;
    std::vector<Cube> cubes;
    std::vector<LevelInfo> levels;
    std::vector<int> leaves;
    // near field: per target leaf, CSR of source ranges
    std::vector<int64_t> p2p_tgt_start, p2p_tgt_end;
    std::vector<int> p2p_ptr;
    std::vector<int64_t> p2p_src_start, p2p_src_end;
    int64_t p2p_pairs = 0;
    // far field
    std::vector<LevelTemplate> tmpl;             // per level
    std::vector<std::vector<M2LPair>> m2l;       // per level
    std::vector<int> m2l_nkeys;                  // per level
    std::vector<std::vector<std::array<int, 4>>> m2l_keyinfo;  // per level, per key: (orbit or -1, offset)
    std::vector<cplx> matpool;                   // all translation matrices
    std::vector<GemvList> m2m_lists, m2l_lists, l2l_lists;  // per level (parent / pair / child level)
    std::vector<M2LTiles> m2l_tiles;                        // per level
    std::vector<M2LChunks> m2l_chunks;                      // per level
    std::vector<LeafTask> s2m_tasks, l2t_tasks;
    int64_t out_total = 0, in_total = 0;         // density array sizes
    int max_s = 0, max_Y = 0, max_Y_leaf = 0;
    // near-field correction tables (built on the device, caller order, blocks of 6)
    bool has_corr = false, has_corr_g = false;
    int64_t corr_blocks = 0;
    // statistics
    std::string stats_json;
    double t_setup_tree = 0, t_setup_tmpl = 0, t_setup_ops = 0, t_setup_corr = 0;
    // device side
    struct Device *dev = nullptr;
};

// set-up stages (host, FP64)
void build_tree(Plan &P);
void build_lists(Plan &P);
void build_templates(Plan &P);
void build_operators(Plan &P);
void build_m2l_tiles(Plan &P, int tile, int chunk);
void build_m2l_chunks(Plan &P, int chunk);
M2LChunks build_chunks(const GemvList &G, int chunk);

// Chunks over the output range [o0, o1) of a list, with the per-pair results
// written to a scratch array (entry order of the list, relative to o0) and
// summed per output in a fixed order afterwards.  Slabs bound the scratch.
std::vector<M2LChunks> build_chunk_slabs(const GemvList &G, int chunk, int64_t max_entries);
void correction_table_host(int64_t n_elem, const double *elem, const double *pts, const double *nrm, const double *w,
                           double k, int op, double coupling, std::vector<int64_t> &rp, std::vector<int64_t> &col,
                           std::vector<cplx> &val);
void nystrom_nodes(int64_t n_elem, const double *elem, double *pts, double *nrm, double *w);
void gauss6(double xi[6][2], double wq[6]);
void p2_shape(double s, double t, double N[6], double dNs[6], double dNt[6]);
void element_eval(const double *el, double s, double t, double y[3], double ys[3], double yt[3]);

// wedge geometry (high-frequency levels)
int wedge_of(const double v[3], int m);
int wedge_neg(int z, int m);
int wedge_child(int z, int m);   // wedge at level with m/2 containing wedge z of level with m
void wedge_center(int z, int m, double c[3]);
WedgeFrame wedge_frame(int z, int m);

}  // namespace fdbem
