// Internal launch interface between the host runtime and the gfx950 kernels.
// Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ra {

// Device block of prices for one evaluation, written by the host before the
// dual kernel runs. F is the problem's element type.  With has_prev set, the
// same pass also returns the lower bound of the previously evaluated prices q:
// the jobs are solved again at q, the used columns are scaled by s (the
// column scales min(1, R_j / r_j) of r(q)) and the scaled utility is summed.
template <typename F>
struct PriceBlock {
    F p[256];     // prices rounded to F
    F invp[256];  // 1 / p_j (+inf where p_j = 0)
    F q[256];     // previous prices
    F invq[256];  // 1 / q_j
    F s[256];     // column scales of r(q)
    F sc[256];    // 1 - s_j, formed in FP64
    int has_prev;
};

// The same prices for the vectorised kernels (m = M), passed by value as a
// kernel argument: no copy to device memory before a pass.
template <int M>
struct PriceArgs {
    float p[M], invp[M], q[M], invq[M], s[M], sc[M];
    int has_prev;
};

// The prices of a small problem's generic solver pass (m <= SMALL_MAX_M),
// passed by value to its one-block kernel (launch_dual_one).
constexpr int SMALL_MAX_M = 64;
constexpr int64_t SMALL_MAX_N = 1024;
template <typename F>
struct SmallPrices {
    F p[SMALL_MAX_M], invp[SMALL_MAX_M], q[SMALL_MAX_M], invq[SMALL_MAX_M], s[SMALL_MAX_M],
        sc[SMALL_MAX_M];
    int has_prev;
};

// Columns of one row of dual-kernel block partials: r_j (m), then the sums of
// net utilities, of scaled utilities U(X~) and of utility lost by scaling.
inline int partial_cols(int m) { return m + 3; }

// One active problem of a batched evaluation (FP32, m in {4, 8, 16, 32}).
// items[n_active] is a sentinel whose tile0 is the total tile count.
constexpr int BATCH_MAX_M = 32;
constexpr int BATCH_COLS = BATCH_MAX_M + 3;  // r_j (padded), net utility, U(X~), loss
// Launch shape of a batched evaluation.  A tile is `rows[c]` consecutive jobs
// of one problem of m class c (m = 4, 8, 16, 32 for c = 0..3): a multiple of
// 64 (one job per lane and step) up to 64 x BATCH_MAX_JPL, holding at most
// `tile_floats` floats of T, the per-wave register budget the kernel is
// compiled for (1024, 2048 or 4096; 1024 only without m = 32 problems).
// Blocks have four waves; `bpc` blocks per compute unit.
constexpr int BATCH_MAX_JPL = 8;
struct BatchShape {
    int tile_floats = 2048;
    int rows[4] = {512, 256, 128, 64};
    int bpc = 0;  // 0: the most that fit
};
__host__ __device__ inline int batch_class(int m) { return m == 4 ? 0 : m == 8 ? 1 : m == 16 ? 2 : 3; }
// LDS row stride of a staged tile row of m floats (padded when m / 4 is even,
// so 16-byte row reads are conflict-free)
__host__ __device__ inline int batch_stride(int m) { return m + (((m >> 2) & 1) ? 0 : 4); }
// True when `rows` is a valid tile height for m under the budget tf.
inline bool batch_rows_ok(int tf, int m, int rows)
{
    return rows >= 64 && rows % 64 == 0 && rows <= 64 * BATCH_MAX_JPL && rows * m <= tf;
}
// A launch shape with the per-job cost of each m class it was measured at
// (ns per job, for the cost-balanced split of the tile space; 0 = not
// measured, the split then weighs 4 m + 8 bytes per job).
struct BatchTuned {
    BatchShape shape;
    double cost[4] = {0.0, 0.0, 0.0, 0.0};
};
struct BatchItem {
    const float* T;      // n x m row-major, 16-byte aligned
    const float2* prm;   // packed (w, c) per job
    int64_t n;
    int m;
    int tile0;           // first tile of this problem in the batch's tile space
    float eps;
    int has_prev;        // the pass also certifies the problem's previous prices
    const float* dem;    // per-job demands, or NULL
    int rows;            // jobs per tile (BatchShape::rows of its m class)
};

// Batched evaluation: k_dual_batch (grid blocks of 4 waves; wave w covers
// tiles [chunk[w], chunk[w+1]) and writes partial slots from segbase[w]) and
// k_batch_reduce (problem a sums slots seg[2a]..seg[2a+1] into out[a][*]).
// prices: per item 6 x BATCH_MAX_M floats (p, 1/p, q, 1/q, s, 1 - s);
// header[0] = number of active items.  lds_floats: LDS floats per wave for a
// staged tile, the largest rows x batch_stride(m) over the batch's m classes.
// Blocks of k_dual_batch compiled for tile budget tf that fit on one compute
// unit with lds_floats per wave.
int batch_blocks_per_cu(int tf, bool demands, bool alpha_fair, int lds_floats);
// With flag (host, fine-grained) and ticket (device counter, zero between
// launches), out is host memory and the launch ends by setting *flag = 1.
hipError_t launch_batch(int tf, int lds_floats, int grid, int max_items, hipStream_t st,
                        const BatchItem* items, const float* prices, const int* chunk,
                        const int* segbase, const int* seg, const int* header, double* partial,
                        double* out, unsigned* ticket = nullptr, unsigned* flag = nullptr,
                        bool demands = false, bool alpha_fair = true);
// Copy `bytes` (a multiple of 16) from pinned, device-visible host memory to
// device memory with a kernel on stream st.
hipError_t launch_copy_table(const void* host_src, void* dst, size_t bytes, hipStream_t st);

// Number of blocks one dual-kernel launch uses for n jobs with m resources
// (dv: with per-job demand vectors).
int dual_grid(int dev_cus, int m, int dtype, int64_t n, bool vec_ok, bool dv = false);

// Dual evaluation (Algorithm 1 per job, sums into block partials).
// partial: [grid][partial_cols(m)] doubles.
// Optional outputs may be null: jpair (n x 2 int16), xpair (n x 2 F),
// tpair (n x 2 F, a_lo x_lo and a_hi x_hi), j1 (n int16).
// dem: per-job scalar demands (n, with w_i / d_i packed in prm); dvec:
// per-job demand vectors (n x m, like T; 16-byte aligned when vec_ok);
// at most one of the two.  prices: the device price block, read by the
// generic kernels; host_prices: the same block in host memory, from which
// the vectorised kernels take their prices as a kernel argument (those need
// no device copy: see dual_is_vec).
hipError_t launch_dual(int dtype, int m, bool vec_ok, int grid, hipStream_t st, const void* T,
                       const void* prm, int64_t n, const void* prices, const void* host_prices,
                       double eps, double* partial, int16_t* jpair, void* xpair, void* tpair,
                       int16_t* j1, const void* dem = nullptr, const void* dvec = nullptr);

// True when launch_dual uses a vectorised kernel (prices as a kernel argument).
bool dual_is_vec(int dtype, int m, bool vec_ok);

// A generic solver pass of a small problem (n <= SMALL_MAX_N, m <=
// SMALL_MAX_M, no demand vectors) as one launch of at most four blocks:
// host_prices is the problem's host price block (PriceBlock of the dtype;
// its first m entries are passed by value), dem the optional per-job
// demands, partial ((n / 256 rounded up) x (m + 3) doubles) and ticket (zero
// between launches) device scratch; the column sums r_j, sum v, sum u(t~),
// sum of the loss go to out (m + 3 doubles of pinned host memory) before
// *flag = 1.
hipError_t launch_dual_small(int dtype, hipStream_t st, const void* T, const void* prm,
                             int64_t n, int m, const void* host_prices, double eps,
                             const void* dem, double* partial, unsigned* ticket, double* out,
                             unsigned* flag);

// Data-dependent starting prices: partial [grid][m] gets, per block, the sums
// of u_i'(a_i^T x) a_ij with x = prices->p (the uniform share of R), each
// term divided by the job's demand for j when dvec (n x m) is given.
hipError_t launch_init(int dtype, int m, bool vec_ok, int grid, hipStream_t st, const void* T,
                       const void* prm, int64_t n, const void* prices, double eps,
                       double* partial, const void* dvec = nullptr);

// out[j] = sum_b partial[b * ncols + j], j < ncols (fixed order).  With flag
// (host memory, fine-grained) and ticket (device counter, zero between
// launches), the launch ends by setting *flag = 1 after every out[j] is
// visible to the host.
hipError_t launch_reduce_cols(hipStream_t st, const double* partial, int nb, int ncols,
                              double* out, unsigned* ticket = nullptr, unsigned* flag = nullptr,
                              const int* skip = nullptr);

// A vectorised dual pass (m in {4, 8, 16, 32, 64}) reading its prices from
// device memory (dprices: a PriceArgs<m> written by the device price loop);
// the pass returns at once when *skip is set.  No per-job outputs.
hipError_t launch_dual_dev(int m, int grid, hipStream_t st, const void* T, const void* prm,
                           int64_t n, double eps, double* partial, const void* dem,
                           const void* dvec, const void* dprices, const int* skip);

struct DevLoop;
struct DevStatus;
// The column sums of a dual pass (partial: nb rows of m + 3) into out, then
// one step of the device price loop (loop.hip), which writes the next pass's
// prices to pa (a PriceArgs<m>) and, when the loop ends, its outcome to hs
// (host memory).  Returns at once when the loop has ended.  m in {4, 8, 16,
// 32, 64}.
hipError_t launch_reduce_step(int m, hipStream_t st, const double* partial, int nb, DevLoop* L,
                              double* out, void* pa, DevStatus* hs);

// Lower bound of the column-scaled allocation (§5): partial2 [grid][2] gets
// sum_i u_i(t~_i) and sum_i u_i(t_i) - u_i(t~_i); r and R are device m-vectors.
int lower_grid(int dev_cus, int64_t n);
hipError_t launch_lower(int dtype, int grid, hipStream_t st, const int16_t* jpair,
                        const void* tpair, const void* prm, int64_t n, int m, const double* R,
                        const double* r, double eps, double* partial2, const void* dem = nullptr);

// Per-job demands: op 0 copies the packed weights into w0; op 1 checks d
// (NULL = all 1) into dem and packs w0 / d; op 2 restores the weights from w0.
hipError_t launch_demands(int dtype, hipStream_t st, int op, const void* d, void* w0, int64_t n,
                          void* prm, void* dem, int* bad);

// Pack (w, c, kind) into one 2-vector per job: (w, c) for capped-linear jobs,
// (w, -1) for log jobs. bad gets bit 1 for w <= 0 / non-finite, bit 2 for a
// bad cap, bit 4 for an unknown kind.
hipError_t launch_pack(int dtype, hipStream_t st, const void* w, const void* c,
                       const uint8_t* kind, int64_t n, void* prm, int* bad);

// bad gets bit 8 if any entry is negative (with positive: not > 0) or
// non-finite.
hipError_t launch_validate_T(int dtype, hipStream_t st, const void* T, int64_t count, int* bad,
                             bool positive = false);

// Dense X~ (n x m, element type F) from the support and column scales.
hipError_t launch_materialize(int dtype, hipStream_t st, const int16_t* jpair, const void* xpair,
                              int64_t n, int m, const double* R, const double* r, void* X);

}  // namespace ra
