// Internal interface between the C ABI (lens_api.hip) and the kernels
// (lens_kernels.hip).  Plain structs of device pointers and host launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lens {

struct PotPtrs {
    int n;
    const double *x, *y, *eps, *phi, *r_core, *r_cut, *sigma_v;
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

constexpr int kTileX = 32, kTileY = 8;  // cells per triangle-stage tile
constexpr int kTriBlocks = 2048;         // persistent workgroups of the triangle stage
constexpr long long kHitScratch = 8192;   // largest hit list sorted in LDS (2^13)
constexpr long long kFlagScratch = 1 << 20;
constexpr int kMaxSystems = 1 << 19;      // systems fit the packed sort key

hipError_t launch_head(const PotPtrs& pot, const GridDesc& g, const ObsPtrs& obs, double* tab64, float* tab32,
                       double* bterm, double* bx, double* by, double* sysrow, EvalState* st, hipStream_t s);
hipError_t launch_field32(const float* tab32, int np, const GridDesc& g, float* ax, float* ay,
                          const EvalState* st, int npl, hipStream_t s);
hipError_t launch_field64(const double* tab64, int np, const GridDesc& g, double* ax, double* ay,
                          const EvalState* st, hipStream_t s);
int tri_blocks(const GridDesc& g);
hipError_t launch_tri32(const float* ax, const float* ay, const GridDesc& g, int nsys, const double* sysrow,
                        EvalState* st, int mode, float tau, unsigned long long* hit_keys, long long hit_cap,
                        unsigned long long* flag_keys, long long flag_cap, unsigned* part, hipStream_t s);
hipError_t launch_tri64(const double* ax, const double* ay, const GridDesc& g, int nsys, const double* sysrow,
                        EvalState* st, unsigned long long* hit_keys, long long hit_cap, unsigned* part,
                        hipStream_t s);

// Outputs and lists of the tail of a chi^2 evaluation.
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

hipError_t launch_fbpos(const double* tab64, int np, const GridDesc& g, const double* sysrow, EvalState* st,
                        const unsigned long long* hit_keys, long long hit_cap, const unsigned long long* flag_keys,
                        long long flag_cap, unsigned long long* fb_keys, long long fb_cap, double* pos,
                        double* fb_pos, hipStream_t s);
hipError_t launch_tail(const TailLaunch& tl, EvalState* st, const unsigned long long* fb_keys, const double* pos,
                       const double* fb_pos, hipStream_t s);
hipError_t launch_dls(double zl, const double* zs, int n, double om, double ol, double* out, hipStream_t s);
hipError_t launch_export(const double* sysrow, int nsys, const EvalState* st, double* bar_x, double* bar_y,
                         int* status, hipStream_t s);

}  // namespace lens
