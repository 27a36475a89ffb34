// Internal interface between the GMRES driver and the network object.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/m1.h"

namespace m1 {

uint16_t* nn_input(m1nn* n);
const float* nn_output(m1nn* n);
int nn_cin_pad(const m1nn* n);
int nn_cin(const m1nn* n);
int nn_cout(const m1nn* n);
int nn_levels(const m1nn* n);
int nn_hmax(const m1nn* n);
int nn_wmax(const m1nn* n);
m1_status nn_run(m1nn* n, int H, int W, hipStream_t s, const int* skip);

// Learned-preconditioner features of a residual r (2D, n_u = 3), written as the
// network input (H x W x cin_pad bf16) or, for training, as FP32 (H x W x cin):
//   [s r/|r| (3), s M^{-1} r/|r| (3), log10(1 + c sigma dt)/4, f_x, f_y],  s = sqrt(3N).
template <typename TV>
void launch_nn_features(int64_t N, const TV* r, const double* rnorm2, const double* bjinv, const double* Uk,
                        const double* sigma, double c, double cdt, int cpad, uint16_t* in_bf16, float* out_f32,
                        hipStream_t s, const int* skip = nullptr);
// z = M^{-1} (r + (|r| / s) y)   (y: network output, H x W x 3)
template <typename TV, typename TZ>
void launch_nn_combine(int64_t N, const TV* r, const double* rnorm2, const double* bjinv, const float* y, TZ* z,
                       hipStream_t s, const int* skip = nullptr);
// training target s (M e - r) / |r|  (H x W x 3, FP32; M the diagonal block)
void launch_nn_target(int64_t N, const double* r, const double* e, const double* rnorm2, const double* bjinv,
                      float* t, hipStream_t s);

}  // namespace m1
