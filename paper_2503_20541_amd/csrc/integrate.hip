// Velocity Verlet (DIMOS Sec. II.D.1): the half kick + drift of steps 1-2 and
// the closing half kick of step 5, with positions wrapped back into [0, L).
#include "mdx_internal.h"

namespace mdx {

__device__ __forceinline__ float wrap_box(float x, float L) {
  if (x >= L) {
    x -= L;
  } else if (x < 0.f) {
    x += L;
    if (x >= L) x = 0.f;   // a tiny negative x rounds onto L
  }
  return x;
}

__global__ void __launch_bounds__(256) k_kick_drift(float* __restrict__ pos,
                                                    float* __restrict__ vel,
                                                    const float* __restrict__ force,
                                                    const float* __restrict__ acc_over_m, int n,
                                                    float half_dt, float dt, float Lx, float Ly,
                                                    float Lz, int* __restrict__ gate) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (gate && a == 0) *gate = 0;
  if (a >= n) return;
  float h = half_dt * acc_over_m[a];
  float L[3] = {Lx, Ly, Lz};
  for (int d = 0; d < 3; ++d) {
    size_t k = (size_t)d * n + a;
    float v = vel[k] + h * force[k];
    vel[k] = v;
    pos[k] = wrap_box(pos[k] + dt * v, L[d]);
  }
}

template <bool ENERGY>
__global__ void __launch_bounds__(256) k_kick(float* __restrict__ vel,
                                              const float* __restrict__ force,
                                              const float* __restrict__ acc_over_m,
                                              const float* __restrict__ mass, int n,
                                              float half_dt, double inv_2acc,
                                              double* __restrict__ partials, int pstride) {
  __shared__ double red[16];
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  double ke = 0.0;
  if (a < n) {
    float h = half_dt * acc_over_m[a];
    double v2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      size_t k = (size_t)d * n + a;
      float v = vel[k] + h * force[k];
      vel[k] = v;
      v2 += (double)v * (double)v;
    }
    ke = (double)mass[a] * v2 * inv_2acc;
  }
  if (ENERGY) {
    double s = block_sum(ke, red);
    if (threadIdx.x == 0) partials[kRowKin * pstride + blockIdx.x] = s;
  }
}

hipError_t launch_kick_drift(Ctx& c, float* pos, float* vel, const float* force, float dt,
                             int* gate) {
  k_kick_drift<<<(c.n + 255) / 256, 256, 0, c.stream>>>(pos, vel, force, c.hdt_scale, c.n,
                                                        0.5f * dt, dt, c.box[0], c.box[1],
                                                        c.box[2], gate);
  return hipGetLastError();
}

hipError_t launch_kick(Ctx& c, float* vel, const float* force, float dt, bool energy) {
  const int nb = (c.n + 255) / 256;
  double inv_2acc = 0.5 / c.accel;
  if (energy)
    k_kick<true><<<nb, 256, 0, c.stream>>>(vel, force, c.hdt_scale, c.mass, c.n, 0.5f * dt,
                                           inv_2acc, c.partials, c.max_blocks);
  else
    k_kick<false><<<nb, 256, 0, c.stream>>>(vel, force, c.hdt_scale, c.mass, c.n, 0.5f * dt,
                                            inv_2acc, c.partials, c.max_blocks);
  return hipGetLastError();
}

}  // namespace mdx
