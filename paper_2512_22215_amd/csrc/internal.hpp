// Internal declarations of the LDU pressure-solve library (gfx950).
//
// Data layout in HBM, per multigrid level:
//  - face form (owner, neighbour, upper, lower: the lduMatrix arrays of
//    paper Sec. 2.1) plus ownStart[i], the first face owned by cell i;
//  - a sliced-ELLPACK copy for the product kernels: rows in slices of 64
//    (one wavefront), slice s holding width_s = max row length in the slice;
//    entry k of row r = 64 s + lane sits at sptr[s] + 64 k + lane, so a
//    wavefront streams 64 consecutive int32 columns and 64 consecutive values
//    per step.  Row entries are column-sorted: the "lower" faces (columns
//    below the row) first, then the "upper" ones.  Padding entries point at
//    their own row with value 0.  val holds A, valT holds A^T at the same
//    positions, so the transposed product runs the same kernel.
//  - levels whose row lengths vary (the Galerkin coarse levels: 3 to ~27
//    entries, which pads max-width slices by 40-50%) use compressed slices:
//    inside each slice of 64 rows the rows are ordered by length (longest
//    first; perm maps a slice position to its row, iperm back), and entry k
//    of lane l is stored at sptr[s] + otab[tptr[s] + k] + l, where
//    otab[tptr[s] + k] counts the entries of the slice's first k columns.
//    Nothing is padded, and a row's loads and stores stay inside the slice's
//    own cache lines.
//  - 16-bit columns: for each stored column k of a slice (a "slot": the k-th
//    entries of the slice's rows), cbase holds the smallest column of the
//    slot and c16 each entry's column minus that base.  Slots that span at
//    most 65535 columns use them in the product kernels (2 bytes per entry
//    instead of 4, and a shorter stream between the reuses of x); wider
//    slots have base -1 and read the 32-bit columns.  A level without any
//    narrow slot keeps c16 = NULL.  The slot of (s, k) is (sptr[s] / 64) + k
//    in plain slices and tptr[s] + k in compressed ones (which keep 32-bit
//    columns).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "ldu.h"

namespace ldu {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaxGrid = 2048;     // streaming kernels: at most this many blocks
// FP64 products on plain slices: at most this many blocks walk slices (the
// rest only contribute zero partials).  Four waves per SIMD instead of eight
// keep fewer of the streamed matrix lines in flight, so more of x survives
// in L2 between its reuses one mesh plane apart.
#ifndef LDU_PLAIN_F64_BLOCKS
#define LDU_PLAIN_F64_BLOCKS 1024
#endif
constexpr int kPlainF64ProductBlocks = LDU_PLAIN_F64_BLOCKS;
#ifndef LDU_CMP_BATCH
#define LDU_CMP_BATCH 24
#endif
constexpr int kCmpBatch = LDU_CMP_BATCH;  // compressed-slice row products: entries per batch
// level-0 vector kernels stream their vectors with nontemporal loads and
// stores above this many cells: four FP64 vectors then exceed the 256 MB
// Infinity Cache, which below it keeps them between kernels
#ifndef LDU_STREAM_NT_CELLS
#define LDU_STREAM_NT_CELLS 12000000
#endif
constexpr int64_t kStreamNtCells = LDU_STREAM_NT_CELLS;
constexpr int kMaxLevels = 64;
constexpr int kMaxCoarseRow = 128; // widest coarse-level row the setup supports
constexpr double kCoarsestTol = 1e-10;
// residual history entries kept on the device per solve (the first ones)
constexpr int64_t kMaxHistory = int64_t(1) << 20;
// largest coarsest level (with off-diagonal entries) the single-workgroup CG
// accepts: its iteration cap max(2n, 100) keeps that kernel to a fraction of
// a second; a hierarchy cut off above it (max_levels, stalled coarsening) is
// refused at setup
constexpr int kMaxCoarsest = 8192;

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void hip_fail(hipError_t e, const char *what, const char *file, int line);
#define HIP_CHECK(x)                                                        \
    do {                                                                    \
        hipError_t e_ = (x);                                                \
        if (e_ != hipSuccess) ::ldu::hip_fail(e_, #x, __FILE__, __LINE__); \
    } while (0)

// ---------------------------------------------------------------- views
template <typename T>
struct SellView {
    int32_t n;
    int64_t nslices;
    const int64_t *sptr;
    const int32_t *col;
    const T *val;
    const T *diag;
    const int32_t *perm;   // row stored at slice position p (NULL: identity)
    const int32_t *iperm;  // slice position of row i (NULL: identity)
    const int32_t *pdeg;   // compressed slices: entries of the row at position p
    const int32_t *tptr;   // compressed slices: start of slice s in otab
    const int32_t *otab;   // compressed slices: offset of entry k within slice s
    const uint16_t *c16;   // column minus its slot base (NULL: use col)
    const int32_t *cbase;  // smallest column of each slot (-1: slot uses col)
};

// scalars shared between the kernels of one solve; device resident
struct DevScalars {
    double rr, bb, rz, rho, pq, alpha, beta, res, bnorm, tol;
    double maxabs, scale;       // mixed: ||r||_inf of the outer residual
    double r0, inner_tol;       // mixed inner CG
    double s;                   // GAMG correction scaling factor
    double inner_now;           // mixed: current inner tolerance
    double mean;                // coarsest: rhs mean
    int iters, max_iter, done, status;
    int inner_iters, inner_max, inner_done;
    int x_pending;              // CG: the iteration's x += alpha p is formed but not yet applied
    unsigned int ticket;        // grid reduction arrival counter (always 0 between kernels)
    unsigned int pad2_;
};

// done codes
enum { kRunning = 0, kConverged = 1, kMaxIter = 2, kFailed = 3 };

// ---------------------------------------------------------------- storage
struct DeviceBuffer {
    void *p = nullptr;
    size_t bytes = 0;
};

class Arena {  // owns every device allocation of a handle
public:
    ~Arena();
    void *alloc(size_t bytes);
    template <typename T>
    T *get(size_t count) { return static_cast<T *>(alloc(count * sizeof(T))); }
    void release(void *p);  // frees one allocation of this arena
    void release_all();

private:
    std::vector<void *> ptrs_;
};

struct Sell {
    int32_t n = 0;
    int64_t nslices = 0, nnz = 0;
    int64_t *sptr = nullptr;
    int32_t *col = nullptr;
    double *val = nullptr, *valT = nullptr;
    float *val32 = nullptr, *valT32 = nullptr;
    double *diag = nullptr;
    float *diag32 = nullptr;
    // compressed slices (levels with uneven rows): lanes sorted by row length
    int32_t *perm = nullptr, *iperm = nullptr, *pdeg = nullptr, *tptr = nullptr, *otab = nullptr;
    // 16-bit column offsets and slot bases (c16 NULL when some slot is too wide)
    uint16_t *c16 = nullptr;
    int32_t *cbase = nullptr;

    __host__ __device__ SellView<double> view(bool transpose) const {
        return {n,    nslices, sptr, col,  transpose ? valT : val, diag, perm, iperm, pdeg,
                tptr, otab,    c16,  cbase};
    }
    __host__ __device__ SellView<float> view32(bool transpose) const {
        return {n,    nslices, sptr, col,  transpose ? valT32 : val32, diag32, perm, iperm, pdeg,
                tptr, otab,    c16,  cbase};
    }
};

// rows stored one after another, each row's entries contiguous and in
// column order (the restriction operators R)
template <typename T>
struct CsrView {
    int32_t n;
    const int64_t *rptr;
    const int32_t *col;
    const T *val;
    int group;  // lanes that share a row in the product kernel
};

struct Csr {
    int32_t n = 0;
    int64_t nnz = 0;
    int64_t *rptr = nullptr;  // [n + 1]
    int32_t *col = nullptr;
    double *val = nullptr, *valT = nullptr;
    float *val32 = nullptr, *valT32 = nullptr;
    int group = 1;
    __host__ __device__ CsrView<double> view(bool transpose) const {
        return {n, rptr, col, transpose ? valT : val, group};
    }
    __host__ __device__ CsrView<float> view32(bool transpose) const {
        return {n, rptr, col, transpose ? valT32 : val32, group};
    }
};

// lanes per row of a CSR product: the power of two nearest the mean row
// length over this many entries per lane, from 1 to 16 (every lane then
// loads its few entries at once, so a long row costs one round trip instead
// of a chain of batches)
#ifndef LDU_CSR_ENTRIES_PER_LANE
#define LDU_CSR_ENTRIES_PER_LANE 2
#endif
constexpr int kCsrEntriesPerLane = LDU_CSR_ENTRIES_PER_LANE;
constexpr int kCsrBatch = 8;  // entries a lane loads before its gathers
// restriction operators with at most this many rows are stored in CSR: there
// a row's lanes load its entries in one round trip.  Above it compressed
// slices win: a lane per row keeps the matrix stream coalesced, and there
// are enough rows to hide the chain of batches
#ifndef LDU_R_CSR_MAX_ROWS
#define LDU_R_CSR_MAX_ROWS 300000
#endif
constexpr int64_t kCsrMaxRows = LDU_R_CSR_MAX_ROWS;

struct Level {
    int32_t n = 0;
    int64_t nf = 0;
    int32_t *own = nullptr, *nb = nullptr;
    double *upper = nullptr, *lower = nullptr, *diag = nullptr;
    int64_t *ownStart = nullptr;          // [n+1]
    int64_t *slotU = nullptr, *slotL = nullptr;  // [nf] positions in the SELL arrays
    Sell A;
    // aggregation to the next level (absent on the coarsest level)
    int32_t nc = 0;
    int32_t *agg = nullptr, *aggStart = nullptr, *aggCells = nullptr;
    // the fine faces each Galerkin sum visits, in its order: per coarse face
    // (cfStart[ncf+1], cfFace: f if the fine owner lies in the coarse owner,
    // else ~f), and per coarse cell its internal fine faces (ciStart, ciFace)
    int64_t *cfStart = nullptr, *ciStart = nullptr;
    int32_t *cfFace = nullptr, *ciFace = nullptr;
    // the down leg of a cycle with one Jacobi pre-sweep from zero as one
    // operator: R = P^T (I - omega A D^-1), a row per coarse cell over this
    // level's columns (valT: the same for A^T), in compressed slices (R) when
    // it has more than kCsrMaxRows rows, else in CSR (Rc)
    Sell R;
    Csr Rc;
    // on a plain-slice level whose R would need compressed slices, the down
    // leg runs over this level's own slices instead: t = (I - omega A D^-1) r
    // with the values -omega a_ij / D_j stored at A's positions (ah; ahT the
    // same for A^T; padding 0), then the member sums of t
    double *ah = nullptr, *ahT = nullptr;
    float *ah32 = nullptr, *ahT32 = nullptr;
    int64_t *r_src = nullptr;             // sources of R's entries, by entry in runs:
    int64_t *r_src0 = nullptr;            //   first source of each entry of R
    int32_t *r_srcn = nullptr;            //   and their count (source -1: a diagonal)
    double r_omega = 0.0;                 // omega the values of R were made for
    bool r_ready = false;                 // R's values match the coefficients
    int singular = 0;                     // coarsest level: A 1 = 0
    int max_row = 0;                      // longest row (off-diagonal entries)
    // V-cycle work vectors
    double *r = nullptr, *e = nullptr, *e2 = nullptr, *t = nullptr;
    float *r32 = nullptr, *e32 = nullptr, *e232 = nullptr, *t32 = nullptr;
    // second ping-pong buffer of the two-stage Gauss-Seidel inner steps
    // (allocated when a cycle asks for three or more of them)
    double *w = nullptr;
    float *w32 = nullptr;
};

}  // namespace ldu

// the opaque handle of the C ABI
struct ldu_t {
    int device = 0;
    bool poisoned = false;
    ldu::Arena arena;            // level-0 and solver buffers
    ldu::Arena gamg_arena;       // hierarchy buffers (rebuilt by gamg_setup)
    ldu::Level L0;
    std::vector<ldu::Level> levels;  // levels[0] aliases L0's arrays when built
    bool gamg_ready = false;
    ldu_gamg_opts gamg_opts{};
    bool f32_ready = false;          // FP32 copies of level values exist
    // solver buffers
    double *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr;
    double *rt = nullptr, *pt = nullptr, *qt = nullptr;  // PBiCG shadow vectors
    float *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *d32 = nullptr;
    double *partials = nullptr;      // [4 * kMaxGrid]
    ldu::DevScalars *dev = nullptr;
    ldu::DevScalars *host = nullptr; // pinned mirror
    double *hist = nullptr;          // device residual history
    int hist_cap = 0;
    int *flag = nullptr;             // device error flag (validation)
    int *hflag = nullptr;            // pinned
    double *coarse_work = nullptr;   // coarsest-level CG scratch (5 n doubles)
    double *dic_dt = nullptr;        // coarsest-level DIC pivots
    bool dic_ready = false;          // dic_dt matches the current coarsest values
    bool dic_ok = false;             // every pivot usable (else diagonal fallback)
};

namespace ldu {

// ---------------------------------------------------------------- launch helpers
inline int stream_grid_slices(int64_t nslices) {
    int64_t g = (nslices + kWavesPerBlock - 1) / kWavesPerBlock;
    if (g > kMaxGrid) g = kMaxGrid;
    if (g >= 64) g &= ~int64_t(7);
    if (g < 1) g = 1;
    return (int)g;
}
inline int64_t slices_of(int64_t n) { return (n + kWave - 1) / kWave; }

// relayout.hip
void build_level_sell(ldu_t *h, Arena &ar, Level &L, bool validate, hipStream_t st);
void set_level_values(Level &L, hipStream_t st);   // face values -> SELL values
void build_sliced_rows(Sell &A, int32_t n, const int32_t *deg, Arena &ar,
                       hipStream_t st);  // compressed slices for given row lengths
void assemble_pressure(ldu_t *h, const double *gamma, const double *w, const double *mag_sf,
                       const double *delta, const double *diag_bc, const double *phi,
                       const double *b_bc, double *b, hipStream_t st);
void ensure_f32(Level &L, Arena &ar, hipStream_t st);
void refresh_f32(Level &L, hipStream_t st);
void exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, Arena &tmp,
                        hipStream_t st);  // out has n+1 entries
void scan_counts_i32(const int32_t *cnt, int32_t *out, int64_t n, Arena &tmp,
                     hipStream_t st);     // out has n+1 entries, int32
void check_finite(ldu_t *h, const double *a, int64_t n, hipStream_t st);

// spmv_pcg.hip
void launch_amul(const SellView<double> &A, const double *x, double *y, hipStream_t st);
void launch_amul32(const SellView<float> &A, const float *x, float *y, hipStream_t st);
void read_scalars(ldu_t *h, hipStream_t st);
void set_scalars_for_solve(ldu_t *h, double tol, int max_iter, hipStream_t st);
double residual_norm(ldu_t *h, const Level &L, bool tr, const double *b,
                     const double *x, double *r_out, hipStream_t st);
int pcg_fp64(ldu_t *h, const double *b, double *x, const ldu_pcg_opts &o,
             bool tr, ldu_stats *stats, hipStream_t st, bool own_hist = true);
int pbicg_fp64(ldu_t *h, const double *b, double *x, const ldu_pcg_opts &o, bool tr,
               ldu_stats *stats, hipStream_t st);
int pcg_mixed(ldu_t *h, const double *b, double *x, const ldu_pcg_opts &o,
              bool tr, ldu_stats *stats, hipStream_t st);
void ensure_hist(ldu_t *h, int64_t entries);
// noalloc.hip: the allocation-free diagonal-PCG entry point's static scratch
constexpr int64_t kNoAllocMaxCells = int64_t(1) << 20;
constexpr int kNoAllocHistory = 4096;
void noalloc_init(int device);
int pcg_fp64_noalloc(ldu_t *h, const double *b, double *x, const ldu_pcg_opts &o,
                     ldu_stats *stats, hipStream_t st);
void copy_history(ldu_t *h, ldu_stats *stats, int count, hipStream_t st);
void launch_coeff_grad(const Level &L, const double *lam, const double *x,
                       double *gd, double *gu, double *gl, hipStream_t st);
void launch_residual_cycle(ldu_t *h, const SellView<double> &A, const double *b,
                           const double *x, double *r, bool maxabs, int grid,
                           hipStream_t st);
void zero_vector(double *a, int64_t n, hipStream_t st);
void launch_residual_plain(ldu_t *h, const SellView<double> &A, const double *b,
                           const double *x, double *r, bool write_hist, int grid,
                           hipStream_t st);
void launch_pcg_q(ldu_t *h, const SellView<double> &A, const double *p, double *q, int grid,
                  hipStream_t st);
void set_done(ldu_t *h, int done, hipStream_t st);
// epilogue after an r update whose partials hold ||r||^2 (and r.z)
void launch_converge(ldu_t *h, int grid, bool with_beta, hipStream_t st);
// x += alpha p (p: the handle's direction) if a stopped CG still owes it
void launch_x_pending(ldu_t *h, double *x, int32_t n, int64_t S, int grid, hipStream_t st);

// gamg.hip
void gamg_build(ldu_t *h, const ldu_gamg_opts &o, hipStream_t st);
void gamg_refresh_values(ldu_t *h, hipStream_t st);
int gamg_fp64(ldu_t *h, const double *b, double *x, const ldu_gamg_opts &o,
              bool tr, ldu_stats *stats, hipStream_t st);
int gamg_mixed(ldu_t *h, const double *b, double *x, const ldu_gamg_opts &o,
               bool tr, ldu_stats *stats, hipStream_t st);
void gamg_vcycle64(ldu_t *h, const double *r, double *e, const ldu_gamg_opts &o,
                   bool tr, hipStream_t st);
int pcg_gamg_fp64(ldu_t *h, const double *b, double *x, const ldu_pcg_opts &o, bool tr,
                  ldu_stats *stats, hipStream_t st);
int pcg_gamg_mixed(ldu_t *h, const double *b, double *x, const ldu_pcg_opts &o, bool tr,
                   ldu_stats *stats, hipStream_t st);
void launch_mx_q(ldu_t *h, const SellView<float> &A32, int G, hipStream_t st);
void launch_mx_update_plain(ldu_t *h, int32_t n, int64_t S, int G, hipStream_t st);
void set_inner(ldu_t *h, double inner_tol, int inner_max, hipStream_t st);
void launch_mx_refine(ldu_t *h, double *x, int32_t n, int64_t S, int G, hipStream_t st);

}  // namespace ldu
