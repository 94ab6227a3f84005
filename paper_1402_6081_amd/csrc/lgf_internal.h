// Internal declarations shared by the library's translation units (not installed).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "lgf_device.h"

namespace lgfdev {

// ------------------------------------------------------------------ constants of the operator
// Level 0 uses the exact lattice Green's function.  Levels >= 1 use it too when the
// interval nodes fall on the lattice (integer node spacing) and max|x_i| < kLatticeRadius;
// everywhere else the far kernel is the asymptotic expansion with kFarTerms terms.
constexpr int kLatticeRadius = 32;
constexpr int kFarTerms = 8;
constexpr int kMaxLevels = 16;

// ------------------------------------------------------------------ launchers (device code)
template <typename T>
hipError_t launch_pad_fft(int m, const T* in, cplx<T>* out, int64_t nbatch, hipStream_t s);
template <typename T>
hipError_t launch_ifft_trunc(int m, const cplx<T>* in, T* out, int64_t nbatch, hipStream_t s);

template <typename T>
hipError_t launch_prod_near(const cplx<T>* fhat, const cplx<T>* khat, const int32_t* nbr, cplx<T>* uhat,
                            int64_t ntarget, int S, hipStream_t s);
template <typename T>
hipError_t launch_prod_far(const cplx<T>* fhat, const cplx<T>* khat, const int32_t* ptr, const int32_t* src,
                           const int32_t* off, cplx<T>* uhat, int64_t ntarget, int S, hipStream_t s);

// Reg block -> level-1 interval: out[b] = (A x A x A) f[b], A is p x n (row-major)
template <typename T>
hipError_t launch_reg_block(const T* f, const double* A, T* out, int64_t nb, int n, int p, hipStream_t s);
// Reg children -> parent: out[J] = sum_c (C_cz x C_cy x C_cx) in[child_c(J)]
template <typename T>
hipError_t launch_reg_up(const T* in, const int32_t* child8, const double* C01, T* out, int64_t nparent, int p,
                         hipStream_t s);
// Interp parent -> children, accumulate: io[c] += (C^T x C^T x C^T) par[parent(c)]
template <typename T>
hipError_t launch_interp_down(const T* par, const int32_t* parent, const int32_t* cpos, const double* C01,
                              T* io, int64_t nchild, int p, hipStream_t s);
// Final: u[b] = vnear[b] + (A^T x A^T x A^T) ut[b], accumulated in FP64 (u may alias vnear)
template <typename T>
hipError_t launch_final(const T* vnear, const T* ut, const double* A, T* u, int64_t nb, int n, int p,
                        hipStream_t s);

// ------------------------------------------------------------------ kernel spectra
struct SpectraKey {
    int n, p, level;   // level 0 = near field
    int radius;        // offsets D in [-radius, radius]^3, id = (Dx+R) + (2R+1)((Dy+R) + (2R+1)(Dz+R))
    int prec;          // 0 = f64, 1 = f32
    bool operator<(const SpectraKey& o) const;
};

struct SpectraEntry {
    SpectraKey key;
    int M = 0, S = 0, noff = 0;
    void* dev = nullptr;  // [noff][S] complex of the plan precision, scaled by 1/M^3
    int64_t bytes = 0;
    ~SpectraEntry();
};

// Get or build the spectra (FP64 generation; rounded to FP32 for prec 1).
std::shared_ptr<SpectraEntry> get_spectra(const SpectraKey& key, hipStream_t s, std::string& err);
int64_t spectra_bytes_total();
void spectra_trim();

// LGF table [R][R][R] (full octant) on the device, FP64, cached per R.
const double* green_table_device(int R, hipStream_t s, std::string& err);
// far kernel A^q at device points (FP64): out[i] = A^q(pts[i])
hipError_t far_kernel_device(const double* pts, int64_t npts, double* out, hipStream_t s, std::string& err);

// ------------------------------------------------------------------ memory accounting
bool budget_reserve(int64_t bytes);
void budget_release(int64_t bytes);
int64_t budget_in_use();
void budget_set(int64_t bytes);

}  // namespace lgfdev
