// Device-resident plan data and the mat-vec / solver launch sequences.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <unordered_map>

#include "plan.hpp"

namespace fdbem {

struct DGemv {
    int n_out = 0, rows = 0, cols = 0, trans = 0, max_rank = 0;
    int64_t n_ent = 0;
    int64_t *out_off = nullptr;
    int *ptr = nullptr;
    int64_t *in_off = nullptr;
    int64_t *mat_off = nullptr;
    int *rank = nullptr;
};

struct DTiles {
    int n_tiles = 0, s = 0, rmax = 1, tile = 0, chunk = 0, nseg = 1;
    size_t shm = 0;
    int64_t *tgt_off = nullptr, *ch_mat = nullptr, *pr_src = nullptr;
    int *tile_ntgt = nullptr, *tile_cptr = nullptr, *ch_rank = nullptr, *ch_pptr = nullptr, *pr_tl = nullptr;
};

struct DChunks {
    int n = 0, s = 0, cols = 0, rmax = 1;
    bool lowrank = false;            // some chunk holds a low-rank (U, V) operator
    size_t shm = 0;
    int64_t *ch_mat = nullptr, *pr_tgt = nullptr, *pr_src = nullptr;
    int *ch_rank = nullptr, *ch_pptr = nullptr;
    // partial-sum schedule: per pair its scratch row, per output its entry range
    int n_out = 0, pw = 16;          // pw: pairs per chunk (16 or 32)
    int64_t n_entries = 0;
    int64_t *pr_pos = nullptr, *red_out = nullptr, *red_ptr = nullptr;
    // wavefront kernel: operator offsets in the row-major pool (null: the workgroup kernel runs)
    int64_t *ch_matw = nullptr;
    int wave_kind = 0;               // operators of the slab: 0 dense, 1 rank <= 16, 2 low-rank, 3 both,
                                     // 4 both and 5 dense with the sources read per row-tile pair
    const double2 *matw = nullptr;
    const float2 *matwf = nullptr;
};

struct DCorr {
    int64_t n_blocks = 0;
    int64_t *rp = nullptr;    // per node: block range
    int32_t *blk = nullptr;   // per block: element (columns 6e .. 6e+5)
    double2 *val = nullptr;   // per block: 6 complex weights
};

struct DBJ {
    int n_blocks = 0, rank = 0;      // rank > 0: learned factors loaded
    int64_t *start = nullptr, *off = nullptr;
    int *size = nullptr;
    double2 *inv = nullptr;          // inverted near-field blocks (column-major n x n at off)
    // overlapping point sets E_b (block points first, caller indices) and the
    // learned factor rows, one row per (block, point of E_b) pair
    int *ne = nullptr;
    int64_t *ext = nullptr;          // n_blocks x 128
    int64_t *poff = nullptr;         // first pair row of each block
    int64_t n_pairs = 0;
    double *O = nullptr;             // network outputs per pair row
};

struct DLearn {
    double2 *T = nullptr;            // targets: column-major n x ne per block at toff
    int64_t *toff = nullptr;
    double *F = nullptr, *H = nullptr, *dout = nullptr, *loss = nullptr;
    double *cw = nullptr;            // per-block weights from the method's GMRES runs (null: 1)
    bool cw_active = false;
};

struct DLeaf {
    int n = 0;
    int n_groups = 0;          // groups of up to L2T_G consecutive tasks of one template
    int *gptr = nullptr;       // group g: tasks [gptr[g], gptr[g + 1])
    int64_t *start = nullptr, *end = nullptr, *slot = nullptr;
    int *tmpl = nullptr;
    double *center = nullptr;  // n x 3
};

struct Device {
    int device = 0;
    // points (sorted order)
    double *x = nullptr, *y = nullptr, *z = nullptr, *nx = nullptr, *ny = nullptr, *nz = nullptr, *w = nullptr;
    int64_t *perm = nullptr;
    void *pn = nullptr;          // packed positions and normals (64 B per point)
    // near field
    int n_leaf = 0;
    int64_t *p2p_ts = nullptr, *p2p_te = nullptr, *p2p_ss = nullptr, *p2p_se = nullptr;
    int *p2p_ptr = nullptr;
    // templates
    int n_lev = 0;
    int *t_s = nullptr, *t_ny = nullptr;
    int64_t *t_yoff = nullptr, *t_woff = nullptr;
    double *t_Y = nullptr;       // concatenated check points
    double2 *t_W = nullptr;      // concatenated W matrices
    double2 *t_Wt = nullptr;     // the same, each transposed (element (r, a) at a + r |Y|)
    // translations
    double2 *mat = nullptr;
    double2 *matw = nullptr;           // row-major operators of the wavefront chunk kernel
    float2 *matwf = nullptr;
    std::unordered_map<int64_t, int64_t> wmap;  // pool offset * 2 + transposed use -> offset in matw
    std::vector<DGemv> m2m, m2l, l2l;  // per level
    std::vector<DTiles> m2lt;          // per level, tiled M2L
    std::vector<DChunks> m2lc;         // per level, operator-chunk M2L
    std::vector<DChunks> m2mc, l2lc;   // per level, operator-chunk M2M and L2L
    // per level, slabs of the partial-sum schedule (default) and its scratch
    std::vector<std::vector<DChunks>> m2ls, m2ms, l2ls;
    void *part = nullptr;
    size_t part_bytes = 0;
    bool part_pipe = false;            // part holds two slab buffers (pipelined slabs)
    void *static_part = nullptr;       // this device's copy of the static scratch
    int m2l_mode = 0;                  // 0 operator chunks, 1 per-target GEMV, 2 target tiles
    double2 *m2l_part = nullptr;       // partial sums of split tiles
    std::vector<std::array<int64_t, 4>> tile_stats;  // per level: tiles, chunks, pairs, segments
    DLeaf s2m, l2t;
    // work vectors
    double2 *dens = nullptr;     // weighted sorted density (N)
    double2 *res = nullptr;      // sorted result (N)
    double2 *od = nullptr, *id = nullptr;
    int prec = 0;                // 0 FP64, 1 FP32 far field and P2P
    float2 *matf = nullptr, *t_Wf = nullptr, *t_Wtf = nullptr, *odf = nullptr, *idf = nullptr;
    int64_t n_od = 0, n_id = 0;
    // near-field corrections (caller order, block CSR: 6 columns per element)
    DCorr corr, corrg;
    DBJ bj;                      // block-Jacobi preconditioner (built on first use)
    DLearn lt;                   // training data of the learned correction
    double2 *gm_z = nullptr, *gm_t = nullptr;
    // GMRES work space (allocated on first solve)
    int gm_m = 0;
    double2 *gm_V = nullptr, *gm_w = nullptr, *gm_x = nullptr, *gm_r = nullptr, *gm_h = nullptr;
    double2 *gm_red_c = nullptr;
    // mat-vecs replayed from captured HIP graphs (keyed by operator and buffers)
    struct GraphEntry {
        hipGraphExec_t exec = nullptr;
        int op = 0;
        const void *in = nullptr;
        void *out = nullptr;
    };
    int use_graph = 0;
    // per tuned (translation, level): level, pairs per chunk, ms(16), ms(32), kind (0 M2L, 1 M2M, 2 L2L),
    // kernel (0 workgroup chunks, 1 wavefront chunks: not tuned)
    std::vector<std::array<double, 6>> autotune;
    size_t mfma_lds = 65536;   // dynamic LDS limit set on the chunk kernels
    hipStream_t cap = nullptr;
    std::vector<GraphEntry> graphs;
    // timing
    int timing = 0;
    static constexpr int kRing = 64;     // timed mat-vecs kept for averaging
    std::vector<hipEvent_t> ev;          // kRing x 10 events, recorded without synchronising
    int ring_pos = 0, ring_count = 0;
    double phase_ms[8] = {0};
    std::vector<void *> allocs;
    size_t bytes = 0;
};

void device_upload(Plan &P);
void device_free(Plan &P);
void device_phase_average(Plan &P);
void build_corrections_device(Plan &P, Device &D);
void build_block_jacobi(Plan &P, Device &D);
void apply_block_jacobi(Plan &P, const double2 *v, double2 *z, hipStream_t st, int mode);
void learned_targets(Plan &P);
int learned_weight_blocks(Plan &P, const double2 *rhs, int iters);

struct LearnedNet;
int learned_num_params();
LearnedNet *learned_create(uint64_t seed);
void learned_destroy(LearnedNet *N);
void learned_set_params(LearnedNet *N, const double *th);
void learned_get_params(LearnedNet *N, double *th);
void learned_get_grad(LearnedNet *N, double *g);
double learned_loss_grad(LearnedNet *N, Plan &P);
double learned_train_step(LearnedNet *N, Plan &P, double lr);
void learned_attach(LearnedNet *N, Plan &P);
void learned_detach(Plan &P);
double learned_loss_grad_raw(LearnedNet *N, int nb, const int64_t *poff, const int *bsize, const int *bne,
                             const int64_t *boff, const int64_t *toff, int64_t n_rows, const double *F,
                             const double2 *Binv, const double2 *T, const double *cw);
void device_matvec(Plan &P, int op, const double2 *in, double2 *out, hipStream_t st, void *part = nullptr);
// size of the file-scope scratch of the allocation-free mat-vec
constexpr size_t kStaticScratchBytes = size_t(256) << 20;
void *static_scratch_address(int device);
void device_matvec_static(Plan &P, int op, const double2 *in, double2 *out, hipStream_t st);
// device_matvec through a captured graph when the plan has graphs enabled
void graph_matvec(Plan &P, int op, const double2 *in, double2 *out, hipStream_t st);
void graph_release(Device &D);

struct Batch;
Batch *batch_create(Plan *const *plans, int n);
void batch_destroy(Batch *B);
void batch_matvec(Batch *B, int op, const double2 *const *in, double2 *const *out, hipStream_t st);
int batch_solve(Batch *B, int op, const double2 *const *rhs, double tol, int maxit, int restart, int precond,
                double2 *const *x, int *iters, double *relres, int *status);
void device_rhs_plane_wave(Plan &P, const double d[3], double2 *rhs, hipStream_t st);
void device_rhs_neumann(Plan &P, const double2 *q, double2 *rhs, hipStream_t st);
int device_gmres(Plan &P, int op, const double2 *b, double tol, int maxit, int restart, int precond, double2 *x,
                 int *iters, double *relres, double *hist, hipStream_t st);

}  // namespace fdbem
