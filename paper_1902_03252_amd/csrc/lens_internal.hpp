// Internal interface between the C ABI (lens_api.hip) and the kernels
// (lens_kernels.hip).  Plain structs of device pointers and host launchers.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lens {

struct PotPtrs {
    int n;
    const double *x, *y, *eps, *phi, *r_core, *r_cut, *sigma_v;
};

// Pseudo-elliptical NFW halos (structure of arrays, device pointers).
struct NfwPtrs {
    int n;
    const double *x, *y, *eps, *phi, *r_s, *kappa_s;
};

struct GridDesc {
    double x0, y0, h;
    int nx, ny;
};

struct ObsPtrs {
    int n_sys, n_img;
    const int* sys_off;
    const double *x, *y, *sigma, *dls;
};

struct EvalState;

// Start/stop events recorded by the dispatch of one kernel itself, so that
// their difference is the kernel's own duration.
struct KernelEvents {
    hipEvent_t start, stop;
};

// Launches `kernel`, timed by `ev` when it is not null.
template <typename F, typename... Args>
inline hipError_t launch_ev(const KernelEvents* ev, F kernel, dim3 grid, dim3 block, hipStream_t s, Args... args)
{
    if (ev)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, ev->start, ev->stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
    return hipGetLastError();
}

// Work plan of one chunk of a batch (device arrays), built on the host.
struct BatchPlan {
    int n;                        // samples in the chunk
    const int* pot_off;           // [n+1] parameter columns of each sample (absolute)
    const GridDesc* grid;         // [n]
    const int* perm;              // [n] plan position -> sample (heaviest first)
    const long long* fitem_off;   // [n+1] field work items, in plan order
    const long long* titem_off;   // [n+1] triangle-stage items (tile row x 64 tile columns), in plan order
    const long long* node_off;    // [n] offset of each sample's field (nodes)
    const long long* rr_off;      // [n] offset of each sample's tile range partials (values)
    int tx_shift;                 // log2 of the tile width in cells
};

// Per-sample counters and status of a batch chunk (device arrays).
struct BatchState {
    unsigned long long* n_hits;   // [n] certain hits
    unsigned long long* n_fb;     // [n] fallback hits
    unsigned long long* n_flags;  // [1] undecided tests of the chunk
    int* status;                  // [n]
};

constexpr long long kHitScratch = 8192;   // largest hit list sorted in LDS (2^13)
constexpr long long kFlagScratch = 1 << 20;
constexpr int kMaxSystems = 1 << 19;      // systems fit the packed sort key
constexpr int kBatchMax = 1024;           // batch: per-sample hit capacity, images and systems

// Arguments of the head's source-plane part when it runs inside a field launch.
struct HeadArgs {
    PotPtrs pot;
    GridDesc g;
    ObsPtrs obs;
    const double* tab64;  // prepared by launch_prep
    const double* bterm;
    double *bx, *by;      // [n_img] grad Psi, then beta
    double* sysrow;
    EvalState* st;
};

hipError_t launch_prep(const PotPtrs& pot, const GridDesc& g, double* tab64, float* tab32, double* bterm,
                       EvalState* st, hipStream_t s);
hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t s);
int fused_head_fits(const GridDesc& g, const ObsPtrs& obs, int npl, bool fp32);
// FP32 field layout code (lens_chi2_opts.field_npl): C = 1, 2, 4 or 8
// consecutive nodes of one row per thread, or 16 R + C for C consecutive nodes
// in each of R consecutive rows (0x21, 0x22, 0x24, 0x41, 0x42).
inline int field_cols(int code) { return code & 15; }
inline int field_rows(int code) { return (code >> 4) ? (code >> 4) : 1; }
inline bool field_code_ok(int code)
{
    return code == 1 || code == 2 || code == 4 || code == 8 || code == 0x21 || code == 0x22 || code == 0x24 ||
           code == 0x41 || code == 0x42;
}
// Layouts of the batched FP32 field (one workgroup per (sample, block of rows,
// row segment)).
inline bool bfield_code_ok(int code)
{
    return code == 1 || code == 2 || code == 4 || code == 0x21 || code == 0x22 || code == 0x41;
}

hipError_t launch_field32h(const float* tab32, int np, const GridDesc& g, float* ax, float* ay, int npl, float* rr,
                           int tx_shift, int tiles_x, const HeadArgs& h, const KernelEvents* ev, hipStream_t s);
hipError_t launch_field64h(const double* tab64, int np, const GridDesc& g, double* ax, double* ay, double* rr,
                           int tx_shift, int tiles_x, const HeadArgs& h, const KernelEvents* ev, hipStream_t s);
hipError_t launch_head(const PotPtrs& pot, const GridDesc& g, const ObsPtrs& obs, double* tab64, float* tab32,
                       double* bterm, double* bx, double* by, double* sysrow, EvalState* st, hipStream_t s);
hipError_t launch_field32(const float* tab32, int np, const GridDesc& g, float* ax, float* ay,
                          const EvalState* st, int npl, float* rr, int tx_shift, int tiles_x,
                          const KernelEvents* ev, hipStream_t s);
hipError_t launch_field64(const double* tab64, int np, const GridDesc& g, double* ax, double* ay,
                          const EvalState* st, double* rr, int tx_shift, int tiles_x, const KernelEvents* ev,
                          hipStream_t s);
constexpr int kRR = 8;                     // values per (row, column group) of the tile range partials
constexpr int kPairBlocks = 512;           // persistent workgroups of the pair kernel
constexpr int kMaxCull = 4096;             // culling waves (64 tiles per round)
int fbpos_blocks(long long n_tiles);       // persistent workgroups of the positions / fallback kernel
void tile_dims(int shape, int& tx, int& ty);
long long tri_tiles(const GridDesc& g, int shape, int* tiles_x);
void cull_shape(const GridDesc& g, int shape, int nsys, int* n_cull, int* tpw, int* sc, int* n_chunks);
hipError_t launch_cull(bool fp32, const void* rr, const GridDesc& g, int nsys,
                       const double* sysrow, unsigned long long* pairs, long long region, unsigned* counts,
                       unsigned* part, int shape, hipStream_t s);
hipError_t launch_pairs(bool fp32, const void* ax, const void* ay, const GridDesc& g, const double* sysrow,
                        EvalState* st, int mode, float tau, const unsigned long long* pairs, long long region,
                        const unsigned* counts, int n_cull, unsigned long long* hit_keys, long long hit_cap,
                        unsigned long long* flag_keys, long long flag_cap, unsigned* part, int part_base, int shape,
                        hipStream_t s);
hipError_t launch_fbpos(const double* tab64, int np, const GridDesc& g, const double* sysrow, EvalState* st,
                        const unsigned long long* hit_keys, long long hit_cap, const unsigned long long* flag_keys,
                        long long flag_cap, unsigned long long* fb_keys, long long fb_cap, double* pos,
                        double* fb_pos, int blocks, hipStream_t s);

// Arguments of the tail kernel.
struct TailLaunch {
    ObsPtrs obs;
    long long hit_cap, flag_cap, fb_cap;
    int hit_capacity;
    const unsigned long long* hit_keys;
    int* out_hits;
    double* img_xy;
    int* n_pred;
    double* contrib;
    double* chi2;
    double* chi2_sys;
    int* match;
    long long* stats;
    long long n_tests;
    const unsigned* part;
    int n_parts;
};

hipError_t launch_tail(const TailLaunch& tl, EvalState* st, const unsigned long long* fb_keys, const double* pos,
                       const double* fb_pos, hipStream_t s);

// Device state of the source-plane chi^2 (zeroed once at allocation).
struct SrcState {
    unsigned ticket;  // "last workgroup" ticket, zero between launches
    int bad;          // a potential outside the model's domain (reset by the last workgroup)
    int status;       // status of the latest forward pass
    int pad;
};

size_t vjp_scratch(int np, const GridDesc& g);  // bytes of device scratch of launch_vjp
hipError_t launch_vjp(const PotPtrs& pot, const GridDesc& g, bool fp32, const double* gx, const double* gy,
                      double* scratch, double* grad, int* status, const KernelEvents* ev, hipStream_t s);
// HMC stages applied by the source-plane gradient kernel to the entries it
// writes: p -= kick * step * grad / 2, then (drift) q += step * p, where
// step != 0.
struct HmcUpdate {
    double* p;
    double* q;
    const double* step;
    double kick;
    int drift;
};

hipError_t launch_src(const PotPtrs& pot, const ObsPtrs& obs, double* beta, double* cot, double* csys,
                      SrcState* st, double* chi2, int* status, const double* g_chi2, double* grad,
                      const HmcUpdate* upd, hipStream_t s);

// Device state of the mixed-precision SIE gradient (reset by its first kernel).
struct MixState {
    unsigned n_list;   // DP list length
    unsigned n_patch;  // list entries that are block pixels
    int status;
    int pad;
};

// Arguments of the mixed-precision SIE gradient.
struct MixedLaunch {
    double* tab64;
    float* tab32;
    double* bterm;
    MixState* st;
    double *ax, *ay;       // [ny*nx] output
    unsigned char* mask;   // [ny*nx] 0 FP32, 1 DP block, 2 DP by the criteria
    unsigned* list;        // [ny*nx] DP pixel list
    long long* stats;      // [4] block pixels, criteria pixels, DP pixels, status
    int n_cluster, pc, pg, npl;
    double t12, t34;
    const KernelEvents* ev;  // times the FP32 field kernel when not null
};

hipError_t launch_mixed(const PotPtrs& pot, const GridDesc& g, const MixedLaunch& ml, hipStream_t s);

size_t nfw_scratch(int np);  // bytes of device scratch of launch_nfw
hipError_t launch_nfw(const NfwPtrs& h, const GridDesc& g, bool fp32, void* ax, void* ay, int* status,
                      void* scratch, const KernelEvents* ev, hipStream_t s);

hipError_t launch_hmc_begin(const double* state, const double* momentum, const double* step, int n7, double* q,
                            double* p, hipStream_t s);
hipError_t launch_hmc_accept(double* state, const double* q, const double* momentum, const double* p,
                             const double* step, int n7, const double* chi2_pair, const int* status_pair,
                             const double* u, double* chi2, int* accepted, hipStream_t s);
hipError_t launch_mh_propose(const double* state, const double* step, const double* noise, int n, int b,
                             double* prop, hipStream_t s);
hipError_t launch_mh_accept(double* state, const double* prop, int n, int b, const double* chi2_new,
                            const int* status_new, const double* u, double* chi2, int* accepted, hipStream_t s);

hipError_t launch_bhead(const BatchPlan& bp, const PotPtrs& pot, const ObsPtrs& obs, double* tab64, float* tab32,
                        double* bterm, double* bx, double* by, int np_chunk, hipStream_t s);
hipError_t launch_bsys(const BatchPlan& bp, const ObsPtrs& obs, const double* bterm, const double* bx,
                       const double* by, double* sysrow, const BatchState& bs, hipStream_t s);
hipError_t launch_bmap(const BatchPlan& bp, int* fmap, int* tmap, hipStream_t s);
hipError_t launch_bfield32(const BatchPlan& bp, const int* fmap, long long n_items, const float* tab32, float* fx,
                           float* fy, float* rr, int npl, const KernelEvents* ev, hipStream_t s);
hipError_t launch_bfield64(const BatchPlan& bp, const int* fmap, long long n_items, const double* tab64, double* fx,
                           double* fy, double* rr, const KernelEvents* ev, hipStream_t s);
hipError_t launch_btri(const BatchPlan& bp, const int* tmap, long long n_items, int nsys, const double* sysrow,
                       const void* fx, const void* fy, const void* rr, bool fp32, const BatchState& bs, int mode,
                       double tau, int hcap, unsigned long long* hits, unsigned long long* flags, long long flag_cap,
                       unsigned* part, int shape, hipStream_t s);
hipError_t launch_bfbpos(const BatchPlan& bp, int nsys, const double* tab64, const double* sysrow,
                         const BatchState& bs, int hcap, const unsigned long long* hits,
                         const unsigned long long* flags, long long flag_cap, unsigned long long* fb, double* pos,
                         double* fb_pos, hipStream_t s);
hipError_t launch_btail(const BatchPlan& bp, const ObsPtrs& obs, const BatchState& bs, int hcap, long long flag_cap,
                        const unsigned long long* hits, const unsigned long long* fb, const double* pos,
                        const double* fb_pos, double* chi2, double* chi2_sys, int* n_pred, int* status,
                        unsigned long long* agg, const unsigned* part, long long n_parts, int* out_nh,
                        int* out_hits, double* out_xy, hipStream_t s);
hipError_t launch_bstats(const unsigned long long* agg, long long n_tests, long long* stats, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
hipError_t launch_dls(double zl, const double* zs, int n, double om, double ol, double* out, hipStream_t s);
hipError_t launch_export(const double* sysrow, int nsys, const EvalState* st, double* bar_x, double* bar_y,
                         int* status, hipStream_t s);

}  // namespace lens
