// Internal declarations shared by the HIP sources of the induced-dipole library.
// Not part of the public ABI (see include/amoeba.h).
#pragma once

#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <cstdint>
#include <string>
#include <vector>

#include "amoeba.h"

namespace amoeba {

constexpr int kBlock = 64;                       // atoms per block = lanes per wave
constexpr double kFixScale = 1099511627776.0;    // 2^40: fixed-point fraction bits of fields
constexpr double kFixInv = 1.0 / 1099511627776.0;
constexpr double kCoulomb = 332.0637133;         // kcal*A/(mol e^2)
constexpr double kDebye = 4.80320;               // D per e*A
constexpr int kBrick = 8;                        // PME spread brick edge (grid points)
constexpr int kMaxFiltered = 2048;               // filtered j-atoms per block (list build)
constexpr int kRedBlocks = 512;                  // workgroups of the deterministic reductions
constexpr double kPi = 3.14159265358979323846;

// Device flags written by validation / preparation kernels.
enum : int {
    kFlagNonFinite = 1,
    kFlagStale = 2,
    kFlagOverflow = 4,
    kFlagBadAlpha = 8,
    kFlagBadThole = 16,
    kFlagBadCsr = 32,
    kFlagFilterOverflow = 64,
    kFlagBreakdown = 128,
    kFlagChanged = 256,
    kFlagBadIndex = 512,
};

// Fixed-point accumulation in FP64 registers and LDS: a contribution v is rounded to the
// nearest multiple of 2^-40 (ties to even) and kept as the integer rint(v * 2^40) in a double.
// Sums of such integers are exact, so they do not depend on the order of the additions
// (FP64 LDS atomics give bitwise-reproducible fixed-point sums), as long as every partial sum
// stays below 2^53 in magnitude, i.e. fields below kFixRange = 2^13 e/A^2; the value is the
// sum times 2^-40.
constexpr double kFixRange = 8192.0;
__device__ __forceinline__ double fixd(float v) { return rint((double)v * 1099511627776.0); }

// LDS sums of the pair and spread kernels: 64-bit integers in units of 2^-38, added with the
// LDS's integer atomics (on gfx950 these measured far faster than its FP64 and FP32 adds).  An
// FP32 value becomes its integer without an FP64-to-integer instruction: adding 1.5 * 2^52 to
// v * 2^38 in FP64 rounds it to the nearest integer (the sum's unit in the last place is 1), and
// the sum's bits minus those of 1.5 * 2^52 are that integer, exact for |v| < 2^13 (the range of
// the fields).  Integer sums are exact, so their order does not matter.
constexpr double kFixQScale = 274877906944.0;      // 2^38
constexpr double kFixQMagic = 6755399441055744.0;  // 1.5 * 2^52
__device__ __forceinline__ unsigned long long fixq(float v)
{
    const double y = fma((double)v, kFixQScale, kFixQMagic);
    return (unsigned long long)(__double_as_longlong(y) - __double_as_longlong(kFixQMagic));
}
// The same for a value already multiplied by 2^38 in FP32 (a power-of-two scaling, exact): the
// widening is exact too, so one FP64 add rounds it exactly as fixq does, to the same integer.
constexpr float kFixQScaleF = 274877906944.0f;    // 2^38
__device__ __forceinline__ unsigned long long fixq_scaled(float vs)
{
    const double y = (double)vs + kFixQMagic;
    return (unsigned long long)(__double_as_longlong(y) - __double_as_longlong(kFixQMagic));
}
__device__ __forceinline__ double fixq_value(unsigned long long q) { return (double)(long long)q * (1.0 / kFixQScale); }

// Sums of an atom's i-field (eipart) and its tile j-fields (jbuf, listed by the reverse index).
// Mixed precision adds every FP32 j-field in the fixed point of the tile accumulators, so the
// sum is exact and does not depend on the order of the reverse-index entries (which the list
// build leaves in the order its atomics gave); FP64 adds the terms as they come, as its tile
// accumulators do.
template <typename R> struct JSum;
template <> struct JSum<float> {
    __device__ static double start(double ei) { return ei * kFixScale; }  // ei: a multiple of 2^-40
    __device__ static double term(float v) { return fixd(v); }
    __device__ static double finish(double a) { return a * kFixInv; }
};
template <> struct JSum<double> {
    __device__ static double start(double ei) { return ei; }
    __device__ static double term(double v) { return v; }
    __device__ static double finish(double a) { return a; }
};

// Workgroups are dispatched round-robin over the eight XCDs (workgroup b runs on XCD b mod 8),
// each with its own L2.  This maps the hardware index to a work item so that every XCD gets a
// contiguous range of items; consecutive items (neighbouring blocks or bricks, which read the
// same atoms and grid points) then share one L2.  A bijection of [0, n).
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    const int q = n >> 3, r = n & 7, x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

// Minimum image used by every FP64 distance decision of the library (list build, in-cutoff
// masks, scaled-pair correction), so that all of them agree bit for bit.
__device__ __forceinline__ double mimg_fp64(double d, double L, double Linv) { return d - L * rint(d * Linv); }

// PCG scalars kept on the device (one struct, FP64).
struct PcgScalars {
    double rzb[2];    // r.z at the start of iteration it, kept in rzb[it & 1]
    double pq;        // p.(A p)
    double gamma;     // step length
    double rz_new;
    double zz;        // z.z -> rms
    double rms;       // rms of z in Debye
    double tol;       // tolerance in Debye
    double epol_acc;  // sum mu.E
    double beta;      // rz_new / rz of the last update
    double rms_sum;   // sum of rms(z) over the iterates since the (re)start: bounds the drift of
                      // the recursive residual (mixed precision)
    int32_t done;     // converged (or broken down): later kernels of the loop skip
    int32_t iters;    // iterations completed
    int32_t status;   // 0 running, 1 converged, 2 breakdown
    int32_t seq;      // direction kernels run since the solve began (publication counter)
    int32_t seq_cur;  // seq and iteration index for the running direction kernel, set by the
    int32_t it_cur;   // update kernel before it (no kernel reads a field it writes)
    int32_t pad[2];
};

// Reduction partials (see reduce.h).
struct RedScratch {
    double* part;
};

struct DeviceBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

}  // namespace amoeba

struct amoeba_ctx {
    amoeba_params prm{};
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;
    int n = 0, nb = 0, npad = 0;
    bool mixed = false;
    bool atoms_set = false;
    bool list_built = false;
    bool cfg_valid = false;        // masks / frames / bins match pos_s
    int64_t n_scaled = 0;
    int ntiles = 0, tile_cap = 0;
    bool skip_mimg = false;        // pair kernels may skip the minimum image (set per list build)
    double* b_extent = nullptr;    // [3] device, flags + 4: largest block half-extent per axis (list build)
    int64_t n_pairs = 0;
    int last_iters = 0;
    double last_rms = 0.0;
    int64_t ws_bytes = 0;

    // allocation registry (freed on destroy)
    std::vector<void*> allocs;

    // sorted-order atom data
    int32_t* perm = nullptr;       // [npad] slot -> original atom (-1 phantom)
    int32_t* slot = nullptr;       // [n] original atom -> slot
    double4* par_d = nullptr;      // [npad] (alpha, 1/alpha, alpha^-1/6, thole)
    double* alpha_s = nullptr;     // [npad] alpha (the PCG preconditioner; 1 on phantom slots)
    double* alpha_inv_s = nullptr; // [npad] 1/alpha (the operator's diagonal)
    float4* par_f = nullptr;       // same in FP32
    int32_t* sc_ptr = nullptr;     // [npad+1] CSR of scaled pairs in slot order
    int32_t* sc_j = nullptr;       // [n_scaled] partner slot
    double* sc_s = nullptr;        // [n_scaled]
    int32_t* sc_ptr_in = nullptr;  // caller-order CSR copy (validation / re-sorting)
    int32_t* sc_j_in = nullptr;
    double* sc_s_in = nullptr;
    // direct-field (d) scales of the same pairs (two-set solve); without them d = p
    bool dscales_set = false;
    int64_t sc_sd_cap = 0;
    double* sc_sd_in = nullptr;    // caller CSR order
    double* sc_sd = nullptr;       // slot order
    double* alpha_in = nullptr;    // caller-order parameters
    double* thole_in = nullptr;

    // per-configuration geometry (slot order)
    double4* pos_s = nullptr;      // [npad] wrapped FP64 positions
    double4* pos_ref = nullptr;    // [npad] positions at the last list build
    double4* blk_org = nullptr;    // [nb] block origin (first atom of the block)
    double4* off_d = nullptr;      // [npad] minimum-image offset from the block origin
    float4* off_f = nullptr;

    // tiles
    int32_t* tile_blk = nullptr;   // [ntiles]
    int32_t* tile_j = nullptr;     // [ntiles*64] j slot or -1
    unsigned long long* tile_mask = nullptr; // [ntiles*64] bit k of row i: pair (i, j_k) within rc
    int32_t* tile_np = nullptr;    // [ntiles] in-cutoff pairs of each tile (per configuration)
    uint16_t* tile_walk = nullptr; // [ntiles*64] first pair of lane l's share of the tile's pairs:
                                   // row | bit << 8, 0xffff for no pairs (per configuration)
    int32_t* tile_rows = nullptr;  // [ntiles] ceil(tile_np / 64): rows of 64 stored pair coefficients
    int32_t* coef_row0 = nullptr;  // [ntiles+1] first stored-coefficient row of each tile (exclusive scan)
    double4* jrel_d = nullptr;     // [ntiles*64] j position relative to the i-block origin
    float4* jrel_f = nullptr;
    int32_t* blk_tile0 = nullptr;  // [nb+1] first tile of each block row

    // PME
    int K[3] = {0, 0, 0};
    int nbr[3] = {0, 0, 0};        // bricks per dimension
    int nbricks = 0;
    size_t ngrid = 0, ncgrid = 0;
    void* grid_r = nullptr;        // real grid (float or double) [K0][K1][K2]
    void* grid_c = nullptr;        // complex half grid [K0][K1][K2/2+1] (plane path: rows padded)
    void* theta_pl = nullptr;      // influence function in the plane path's column-chunk layout
    void* theta = nullptr;         // influence function on the half grid (float or double)
    int32_t* bin_start = nullptr;  // [nbricks+1] atoms binned by the brick of their base point
    int32_t* bin_atoms = nullptr;  // [npad]
    int32_t* bin_count = nullptr;  // [nbricks]
    int32_t* atom_bin = nullptr;   // [npad]
    int4* sp_base = nullptr;       // [npad] base grid point of each atom (x, y, z, real atom)
    void* sp_w = nullptr;          // [npad][32] (R) B-spline weights m0, m1 per dimension
    // dipole reciprocal field by x-planes (plane.hip), used when the grid fits (plane_ok)
    bool plane_ok = false;
    int pme_path = 0;              // amoeba_pme_path requested by the caller
    bool rec_plane = false;        // the last reciprocal field came from the plane path
    bool brick_bins_stale = true;  // brick bins and spline table not built for the current positions
    int32_t* xb_start = nullptr;   // [K0+1] atoms binned by the x line of their base point
    int32_t* xb_count = nullptr;   // [K0+1]
    int4* xb_rec = nullptr;        // [npad] per binned atom: (slot, fx, fy, fz)
    void* xb_w = nullptr;          // [npad] (R4) spline arguments (wx, wy, wz, 0)
    void* rec_part = nullptr;      // [5][npad] (R4) field share of each of an atom's five x-planes
    void* pl_roots[3] = {nullptr, nullptr, nullptr};  // roots of unity exp(-2 pi i m / K) (R complex)
    int npq = 0;                   // p.q partials written by the last PCG product
    int npq_cap = 0;               // room for them at the start of red.part
    rocfft_plan plan_fwd = nullptr, plan_bwd = nullptr;
    rocfft_execution_info exec_fwd = nullptr, exec_bwd = nullptr;
    void* fft_work = nullptr;
    size_t fft_work_bytes = 0;

    // real-space field pieces and vectors (slot order, FP64 N x 3 unless noted)
    double* eipart = nullptr;              // [npad*3] field at i summed over its own block's tiles
    // stored radial coefficients (B1', B2') of every in-cutoff pair: recorded by the first dipole
    // product of a configuration, replayed by the later ones; row r, lane l at r*64 + l (R2)
    int pair_store = 0;                    // amoeba_pair_store requested by the caller
    void* coef = nullptr;                  // [coef_cap_rows*64] (R2)
    int64_t coef_cap_rows = 0;
    int64_t coef_bytes = 0;
    bool coef_ready = false;               // coef holds the current configuration's coefficients
    bool coef_rows_ok = false;             // coef_row0 holds the current tiles' rows
    bool coef_rows_pending = false;        // flags_host[10] receives the row total of the last refresh
    bool coef_last_stored = false;         // the last dipole product stored or replayed every tile
    void* jbuf = nullptr;                  // [tile_cap*64][4] (R) j-field (x, y, z, 0) of every off-diagonal tile slot
    int32_t* rev_ptr = nullptr;            // [npad+1] reverse index: jbuf slots where an atom is j
    int32_t* rev_idx = nullptr;            // [rev_cap] entries tile*64 + lane
    int64_t rev_cap = 0;
    double* ereal = nullptr;               // [npad*3] reduced real-space field
    double* erec = nullptr;                // [npad*3] reciprocal field scratch
    double* v_mu = nullptr;
    double* v_r = nullptr;
    double* v_p = nullptr;
    double* v_q = nullptr;
    double* v_e = nullptr;                 // E_perm in slot order
    double4* pv_d = nullptr;               // [npad] pair-kernel copy of the direction (FP64)
    float4* pv_f = nullptr;                // [npad] (FP32)
    double4* mp_d = nullptr;               // [npad*3] (q,dx,dy,dz),(Txx,Txy,Txz,Tyy),(Tyz,Tzz,0,0)
    float4* mp_f = nullptr;                // same in FP32 (mixed mode)
    void* f_src = nullptr;                 // [npad*4] (R4) multipoles + dipoles of the gradient tiles
    void* f_psi = nullptr;                 // [K0*K1*K2] (R) grid potential of the multipoles (gradient)

    amoeba::PcgScalars* sc = nullptr;      // device scalars
    amoeba::PcgScalars* sc_host = nullptr; // pinned mirror [2] (one per in-flight PCG iteration)
    amoeba::PcgScalars* sc_host_dev = nullptr; // its device-side address
    unsigned long long* pairs_host = nullptr;     // pinned: in-cutoff pair count of the last refresh
    unsigned long long* pairs_host_dev = nullptr; // its device-side address
    amoeba::RedScratch red{};
    int* flags = nullptr;                  // device error flags and list-build status words [256]
    int* flags_host = nullptr;             // pinned
    unsigned long long* pair_part = nullptr; // per-workgroup pair counts of the mask refresh
    bool pairs_pending = false;            // pairs_host receives a pair count (ev_pairs) not yet in n_pairs
    int pair_nwg = 0;                      // pair_part entries of the last mask refresh
    hipEvent_t ev[2] = {nullptr, nullptr};
    // the real-space tiles of a PCG product run on a second stream (default priority), beside
    // the reciprocal passes on the context stream: forked and joined with events
    hipStream_t stream2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_pairs = nullptr;         // recorded after the pair count of a refresh is written
    // one PCG iteration (product on both streams, update, direction) as a HIP graph: captured on
    // gstream, replayed on the context stream; recaptured when a launch parameter it bakes in
    // changes (key).  Off unless the caller asks: measured slower than the direct launches.
    bool use_graphs = false;
    int residual_check = AMOEBA_RESIDUAL_CHECK_AUTO;  // amoeba_residual_check
    hipStream_t gstream = nullptr;
    hipGraph_t it_graph = nullptr;
    hipGraphExec_t it_exec = nullptr;
    unsigned long long it_key = 0;
    int pcg_seq = 0;                       // direction kernels enqueued since the solve began

    // list-build scratch, kept between builds
    unsigned* b_keys = nullptr;            // [n] sort keys (column | x)
    unsigned* b_keys2 = nullptr;           // [n] sorted keys
    int* b_vals = nullptr;                 // [n] atom indices
    int* b_vals2 = nullptr;                // [n] atom indices in key order
    void* b_sort_tmp = nullptr;            // radix sort scratch
    size_t b_sort_bytes = 0;
    double4* b_bc = nullptr;               // [nb] block box centres
    double4* b_bh = nullptr;               // [nb] block box half-extents
    int* b_cell_start = nullptr;           // [b_ncell_cap + 1] first entry of each cell (block grid)
    int b_ncap[3] = {1, 1, 1};             // largest block-grid cell count per axis
    int b_ncell_cap = 0;                   // their product
    int* b_rowc = nullptr;                 // [nb] filtered j count per block
    int* b_rowj = nullptr;                 // [nb * kMaxFiltered]
    int* b_tpb = nullptr;                  // [nb + 1] tiles per block
    int* b_cnt = nullptr;                  // [npad + 1] per-slot counts
    int* rev_cnt = nullptr;                // [npad + 1] reverse-index counters, zero between builds
    int* b_scan = nullptr;                 // [npad / 1024 + 2] scan block sums / offsets

    // learned initial guess (guess.hip); allocated by the first amoeba_guess_set_model
    bool guess_loaded = false;
    float* g_model = nullptr;              // [NMODEL] parameters + mean + inv_std
    float* g_adam_m = nullptr;             // [NPARAM] Adam first moment
    float* g_adam_v = nullptr;             // [NPARAM] Adam second moment
    int64_t g_step = 0;                    // Adam steps taken since the model was set
    float* g_part = nullptr;               // [kGuessWG][NPARAM] per-workgroup gradient partials
    double* g_lossp = nullptr;             // [kGuessWG] per-workgroup loss partials
    double* g_scal = nullptr;              // [4] device scalars (loss)
    double* g_scal_host = nullptr;         // pinned mirror
    double* g_npart = nullptr;             // [kRedBlocks][NFEAT] normalisation partials
    double* g_nmean = nullptr;             // [NFEAT]
    double* g_v = nullptr;                 // [3][npad*3] bases v0, v1, v2 (slot order, FP64)
    double* g_radial = nullptr;            // [npad*3] radial neighbour sums
    float* g_feat = nullptr;               // [npad][NFEAT]
    float* g_basis = nullptr;              // [npad][NBASIS*3]
    double* g_save_mu = nullptr;           // [npad*3] fallback guess kept while the starts are compared
    double* g_save_q = nullptr;            // [npad*3] its A mu0
    void* g_scratch = nullptr;             // this device's address of the no-allocation scratch array
    int g_kind = AMOEBA_GUESS_KIND_NEUMANN; // which bases the network combines
    double* g_ref = nullptr;               // [2][n*3] reference dipoles and field (caller order)
    bool g_ref_set = false;
    int last_guess = 0;
    double last_guess_rms[2] = {0.0, 0.0};

    // stage timing (diagnostic)
    bool timing = false;           // stage timing with the stages one after the other
    bool timing_live = false;      // stage timing with the streams as they are
    std::vector<hipEvent_t> tev;                 // event pool
    std::vector<std::pair<int, int>> trec;       // (stage, index of start event in the pool)
    int64_t matvecs = 0;
};

namespace amoeba {

// allocation helpers (api.hip)
int ctx_alloc(amoeba_ctx* c, void** p, size_t bytes);
int set_error(amoeba_ctx* c, int code, const std::string& msg);
int hip_check(amoeba_ctx* c, hipError_t e, const char* what);

// RAII stage timer: records a start/stop event pair on the context stream when timing is on.
struct StageTimer {
    amoeba_ctx* c;
    hipStream_t st;
    int idx = -1;
    StageTimer(amoeba_ctx* ctx, int stage, hipStream_t stream = nullptr);  // null: context stream
    ~StageTimer();
};

// blocklist.hip
// exclusive, out[n] = total; total_copy: a second place for the total
int device_scan(amoeba_ctx* c, int n, const int* in, int* out, int* total_copy = nullptr);
void coef_scan_rows(amoeba_ctx* c);       // rows of the coefficient store for the current masks
void launch_sum_pairs(amoeba_ctx* c);     // pair count of the last mask refresh into pairs_host
int build_blocklist(amoeba_ctx* c, const double* pos);
int prepare_config(amoeba_ctx* c, const double* pos);

// realspace.hip
void launch_mutual_tiles(amoeba_ctx* c, bool use_done, hipStream_t st = nullptr);  // null: context stream
void iteration_graph_release(amoeba_ctx* c);  // drop the captured PCG iteration
void coef_invalidate(amoeba_ctx* c);      // pair coefficients must be recorded again
int coef_reserve(amoeba_ctx* c);          // size the coefficient store (host has synchronized)
void coef_release(amoeba_ctx* c);         // free it (other allocations come first under the cap)
bool coef_store_on(const amoeba_ctx* c);  // the requested mode uses the store
int next_coef_mode(const amoeba_ctx* c);  // the next dipole product: 0 evaluates, 1 records, 2 replays
void launch_real_reduce(amoeba_ctx* c, double* ereal, hipStream_t st = nullptr, bool use_done = false);
void launch_perm_tiles(amoeba_ctx* c, hipStream_t st = nullptr);
void launch_perm_assemble(amoeba_ctx* c, double* out_slot, const double* scales);  // scales in slot order
void launch_force_tiles(amoeba_ctx* c, const void* src, double* out);  // real-space gradient pair sums

// pme.hip
int pme_setup(amoeba_ctx* c);
void pme_bin_atoms(amoeba_ctx* c);
int pme_dipole_field(amoeba_ctx* c, bool use_done);   // spread p -> FFT -> convolve -> FFT
int pme_perm_potential(amoeba_ctx* c);                // spread multipoles -> ... -> potential grid
void pme_scan_excl(amoeba_ctx* c, int n, const int* in, int* out);

// plane.hip
bool plane_eligible(const amoeba_ctx* c);
int plane_row_stride(const amoeba_ctx* c);  // row stride of the plane path's half grid (complex values)
void plane_column_chunks(const amoeba_ctx* c, int* kc, int* nkc);  // its column chunks (width, count)
int plane_setup(amoeba_ctx* c);
int plane_bin_atoms(amoeba_ctx* c);
void plane_dipole_field(amoeba_ctx* c, bool use_done, int parts);  // 1 spread, 2 the rest, 3 all
void plane_perm_field(amoeba_ctx* c);                             // permanent multipoles, all passes
void plane_gather(amoeba_ctx* c, double* out);          // E_rec from the plane shares
int plane_combine(amoeba_ctx* c, bool use_done, bool dot_pq, bool reduced);  // PCG product; returns its partial count
bool pme_use_planes(const amoeba_ctx* c);
void launch_gather(amoeba_ctx* c, double* out);       // E_rec at atoms from the potential grid
int pme_brick_potential(amoeba_ctx* c, bool perm);    // psi of the multipoles (perm) or of pv, brick path

// force.hip
int polar_gradient_slot(amoeba_ctx* c);               // dE_pol/dr (slot order) into v_q

// api.hip
int read_flags(amoeba_ctx* c, int* out);
int check_vec_finite(amoeba_ctx* c, const double* v, size_t n, const char* what);
void launch_check_overflow(amoeba_ctx* c, const double* v_slot);  // |v| < kFixRange, flag on the device
int begin_config(amoeba_ctx* c, const double* pos, const char* who);

// guess.hip
int guess_compute(amoeba_ctx* c);                     // bases + features of v_e (slot order)
int guess_scratch_init(amoeba_ctx* c);                // device address of the no-allocation scratch
void guess_forward_slot(amoeba_ctx* c, double* mu_slot);

// pcg.hip
void launch_gather_vec(amoeba_ctx* c, const double* src_caller, double* dst_slot);
void launch_scatter(amoeba_ctx* c, const double* v_slot, double* out_caller);
void launch_matvec_combine(amoeba_ctx* c, bool use_done, bool dot_pq, bool reduced = false);  // reduced: E_real already in ereal
void launch_set_direction(amoeba_ctx* c, const double* src);
void launch_gather_vec_checked(amoeba_ctx* c, const double* src_caller, double* dst_slot); // + NaN flag
int pcg_solve(amoeba_ctx* c, double tol, int max_iter, bool have_guess, double* mu_out, double* e_pol);
int pcg_dot_mu_e(amoeba_ctx* c, double* acc);                      // sum of v_mu . v_e (waits)
void pcg_begin(amoeba_ctx* c, double tol);                         // initial device scalars
int pcg_start(amoeba_ctx* c, bool have_guess, double* rms_debye);   // r0, z0, p0 from v_mu
int pcg_start_from(amoeba_ctx* c, const double* q0);                // same, A mu0 given
int pcg_run(amoeba_ctx* c, int max_iter, int start_matvecs, double* mu_out, double* e_pol);
int matvec_slot(amoeba_ctx* c, bool use_done, bool dot, hipEvent_t fork_ev = nullptr);  // q = A p

}  // namespace amoeba
