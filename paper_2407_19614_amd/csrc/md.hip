// Born-Oppenheimer molecular dynamics of the nuclei (the paper's AIMD
// wrapper, NVE): velocity-Verlet half steps and the kinetic energy on device
// arrays, so a dynamics loop keeps positions, velocities and forces in HBM.
#include "kernels.h"

namespace {

// v += (dt/2) a with a = -grad / m; then, for stage 0, x += dt v
__global__ void verlet_kernel(int n, double dt, const double* __restrict__ mass, const double* __restrict__ grad,
                              double* __restrict__ xyz, double* __restrict__ vel, int stage) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 3 * n) return;
    const double v = vel[e] - 0.5 * dt * grad[e] / mass[e / 3];
    vel[e] = v;
    if (stage == 0) xyz[e] += dt * v;
}

// one workgroup: out = sum_a 1/2 m_a |v_a|^2 (fixed summation order)
__global__ __launch_bounds__(256) void kinetic_kernel(int n, const double* __restrict__ mass,
                                                      const double* __restrict__ vel, double* __restrict__ out) {
    double s = 0.0;
    for (int e = threadIdx.x; e < 3 * n; e += 256) s += 0.5 * mass[e / 3] * vel[e] * vel[e];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
    __shared__ double part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = (part[0] + part[1]) + (part[2] + part[3]);
}

int32_t hip_fail(hipError_t e) {
    ri::set_hip_error(hipGetErrorString(e));
    return RI_E_HIP;
}

}  // namespace

extern "C" {

int32_t ri_md_verlet(int32_t n_atoms, double dt, const double* mass, const double* grad, double* xyz, double* vel,
                     int32_t stage, hipStream_t st) {
    if (n_atoms <= 0 || !(dt > 0.0) || !mass || !grad || !xyz || !vel || (stage != 0 && stage != 1)) return RI_E_ARG;
    verlet_kernel<<<(3 * n_atoms + 255) / 256, 256, 0, st>>>(n_atoms, dt, mass, grad, xyz, vel, stage);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RI_OK : hip_fail(e);
}

int32_t ri_md_kinetic(int32_t n_atoms, const double* mass, const double* vel, double* ekin, hipStream_t st) {
    if (n_atoms <= 0 || !mass || !vel || !ekin) return RI_E_ARG;
    kinetic_kernel<<<1, 256, 0, st>>>(n_atoms, mass, vel, ekin);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RI_OK : hip_fail(e);
}

}  // extern "C"
