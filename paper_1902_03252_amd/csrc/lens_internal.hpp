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

constexpr int kTileX = 64, kTileY = 16;  // cells per triangle-stage tile
constexpr long long kHitScratch = 8192;   // largest hit list sorted in LDS
constexpr long long kFlagScratch = 1 << 20;

hipError_t launch_prep(const PotPtrs& pot, const GridDesc& g, double* tab64, float* tab32, double* bterm,
                       hipStream_t s);
hipError_t launch_src(const double* tab64, int np, const ObsPtrs& obs, double* bx, double* by, hipStream_t s);
hipError_t launch_bound(const double* bterm, int np, const GridDesc& g, const ObsPtrs& obs, const double* bx,
                        const double* by, double* sysrow, EvalState* st, hipStream_t s);
hipError_t launch_field32(const float* tab32, int np, const GridDesc& g, float* ax, float* ay,
                          const EvalState* st, int npl, hipStream_t s);
hipError_t launch_field64(const double* tab64, int np, const GridDesc& g, double* ax, double* ay,
                          const EvalState* st, hipStream_t s);
hipError_t launch_tri32(const float* ax, const float* ay, const GridDesc& g, int nsys, const double* sysrow,
                        EvalState* st, int mode, float tau, unsigned long long* hit_keys, long long hit_cap,
                        unsigned long long* flag_keys, long long flag_cap, hipStream_t s);
hipError_t launch_tri64(const double* ax, const double* ay, const GridDesc& g, int nsys, const double* sysrow,
                        EvalState* st, unsigned long long* hit_keys, long long hit_cap, hipStream_t s);
hipError_t launch_fb(const double* tab64, int np, const GridDesc& g, const double* sysrow, EvalState* st,
                     const unsigned long long* flag_keys, long long flag_cap, unsigned long long* hit_keys,
                     long long hit_cap, hipStream_t s);
hipError_t launch_sort(unsigned long long* hit_keys, EvalState* st, long long flag_cap, int hit_capacity, int nsys,
                       int* out_hits, int* n_pred, hipStream_t s);
hipError_t launch_pos(const double* tab64, int np, const GridDesc& g, const double* sysrow, const EvalState* st,
                      int hit_capacity, const unsigned long long* hit_keys, double* img_xy, hipStream_t s);
hipError_t launch_chi2(const ObsPtrs& obs, const EvalState* st, int hit_capacity,
                       const unsigned long long* hit_keys, const double* img_xy, double* contrib, double* chi2,
                       double* chi2_sys, int* match, long long* stats, long long n_tests, hipStream_t s);
hipError_t launch_dls(double zl, const double* zs, int n, double om, double ol, double* out, hipStream_t s);
hipError_t launch_export(const double* sysrow, int nsys, const EvalState* st, double* bar_x, double* bar_y,
                         int* status, hipStream_t s);

}  // namespace lens
