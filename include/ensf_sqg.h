/*
 * ensf_sqg.h -- C ABI of the GPU surface quasi-geostrophic (nonlinear Eady) model in
 * libensf.so: the physics-based forecast model of the paper's twin experiments
 * (Sec. II-B), pseudo-spectral in FP64.
 *
 * Nondimensional units f = N = H = 1 (lengths in Rossby radii), doubly periodic square
 * domain of side lx on an n x n grid, basic flow U(z) = shear (z - 1/2), zero interior
 * potential vorticity.  Per level i (0 = ground, 1 = lid):
 *     d theta_i/dt + (U_i + u_i) d theta_i/dx + v_i (d theta_i/dy - shear) = D(theta_i),
 *     u = -d psi/dy, v = d psi/dx,
 *     psi_0 = -theta_0/(K tanh K) + theta_1/(K sinh K),
 *     psi_1 = -theta_0/(K sinh K) + theta_1/(K tanh K),
 * with the nonlinear term computed on the grid and transformed back with the 2/3 rule on
 * both wavenumber components, classical RK4 in time, and two linear damping terms applied
 * exactly after each step: hyperdiffusion and a thermal relaxation of theta toward the
 * basic state with time scale relax_time (it lets the turbulence equilibrate):
 *     theta_hat *= exp(-dt/efold * (K / (2/3 K_max))^order - dt/relax_time).
 * The FFTs are hipFFT (D2Z / Z2D); everything else runs in this library's kernels.
 *
 * States are (batch, 2, n, n) row-major (component e = level*n*n + iy*n + ix), the layout
 * of one ensemble member of the analysis.  Pointers named d_* are device pointers owned by
 * the caller; calls are stream-ordered on the given stream (hipStream_t as void*).
 */
#ifndef ENSF_SQG_H
#define ENSF_SQG_H

#include <stdint.h>

#include "ensf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ensf_sqg ensf_sqg;

/* n: even grid size >= 8; lx > 0; dt > 0; diff_order >= 2; diff_efold > 0 (e-folding time
   of the highest retained wavenumber, INFINITY = no diffusion); relax_time > 0 (INFINITY =
   no relaxation); max_batch >= 1 states per internal chunk.  device: HIP ordinal. */
ensf_status ensf_sqg_create(int32_t n, double lx, double shear, double dt, int32_t diff_order,
                            double diff_efold, double relax_time, int32_t max_batch,
                            int32_t device, ensf_sqg** out);

/* Advances `batch` FP64 states by n_steps time steps (d_out may equal d_in). */
ensf_status ensf_sqg_run(ensf_sqg* s, const double* d_in, double* d_out, int32_t batch,
                         int32_t n_steps, void* stream);

/* Same for FP32 states (converted to FP64 internally, rounded back at the end). */
ensf_status ensf_sqg_run_f32(ensf_sqg* s, const float* d_in, float* d_out, int32_t batch,
                             int32_t n_steps, void* stream);

/* Frees the model.  NULL is a no-op. */
ensf_status ensf_sqg_destroy(ensf_sqg* s);

#ifdef __cplusplus
}
#endif
#endif /* ENSF_SQG_H */
