// Reciprocal-space Ewald sum evaluated directly over the reciprocal vectors
// (Sec. II.A.2, Eqs. 9-12 with Eq. 11 in its standard form): the O(N^{3/2})
// high-accuracy path beside smooth PME. With m = (n1/L1, n2/L2, n3/L3),
// |n_d| <= n_max, m != 0,
//   S(m) = sum_j q_j exp(2 pi i m.r_j),
//   E    = k_e / (2 pi V) sum_m f(m) |S(m)|^2,  f(m) = exp(-pi^2 m^2/alpha^2) / m^2,
//   F_i  = (2 k_e q_i / V) sum_m f(m) m Im(conj(S(m)) exp(2 pi i m.r_i)).
// Only half of the vectors are visited (m and -m contribute equally). All
// sums are FP64; the per-atom phase factors exp(2 pi i n_d x_d / L_d) are
// tabulated once per call.
//
// k_ew_tables: per atom and axis, the 2 n_max + 1 phase factors.
// k_ew_structure: one block per half-space vector (lexicographically after
//   0), the structure factor and its energy term in fixed order.
// k_ew_forces: one thread per atom, all half-space vectors in the same order.
// k_ew_energy: fixed-order sum of the energy terms.
#include "mdx_internal.h"

namespace mdx {

constexpr int kEwThreads = 256;

__global__ void k_ew_tables(const float* __restrict__ pos, int n, double3 L, int nmax,
                            double2* __restrict__ tab) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * n) return;
  const int d = t / n, a = t - d * n;
  const double Ld = d == 0 ? L.x : (d == 1 ? L.y : L.z);
  const double u = 2.0 * (double)pos[(size_t)d * n + a] / Ld;   // phase / pi for n_d = 1
  const int w = 2 * nmax + 1;
  for (int k = -nmax; k <= nmax; ++k) {
    double s, c;
    sincospi((double)k * u, &s, &c);
    tab[((size_t)d * w + (k + nmax)) * n + a] = make_double2(c, s);
  }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// (n1, n2, n3) of half-space vector h: the cube index h + (w^3 + 1) / 2.
__device__ __forceinline__ void ew_decode(int h, int nmax, int& n1, int& n2, int& n3) {
  const int w = 2 * nmax + 1;
  const int f = h + (w * w * w + 1) / 2;
  n1 = f / (w * w) - nmax;
  n2 = (f / w) % w - nmax;
  n3 = f % w - nmax;
}

__global__ void __launch_bounds__(kEwThreads) k_ew_structure(const double2* __restrict__ tab,
                                                             const float* __restrict__ q, int n,
                                                             int nmax, double3 L, double pi2_a2,
                                                             double2* __restrict__ S,
                                                             double* __restrict__ eterm) {
  __shared__ double sre[kEwThreads], sim[kEwThreads];
  const int h = blockIdx.x;
  int n1, n2, n3;
  ew_decode(h, nmax, n1, n2, n3);
  const int w = 2 * nmax + 1;
  const double2* t1 = tab + (size_t)(0 * w + n1 + nmax) * n;
  const double2* t2 = tab + (size_t)(1 * w + n2 + nmax) * n;
  const double2* t3 = tab + (size_t)(2 * w + n3 + nmax) * n;
  double re = 0.0, im = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double2 e = cmul(cmul(t1[j], t2[j]), t3[j]);
    const double qj = (double)q[j];
    re += qj * e.x;
    im += qj * e.y;
  }
  sre[threadIdx.x] = re;
  sim[threadIdx.x] = im;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sre[threadIdx.x] += sre[threadIdx.x + o];
      sim[threadIdx.x] += sim[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mx = n1 / L.x, my = n2 / L.y, mz = n3 / L.z;
    const double m2 = mx * mx + my * my + mz * mz;
    const double f = exp(-pi2_a2 * m2) / m2;
    S[h] = make_double2(sre[0], sim[0]);
    eterm[h] = f * (sre[0] * sre[0] + sim[0] * sim[0]);
  }
}

__global__ void __launch_bounds__(kEwThreads) k_ew_forces(const double2* __restrict__ tab,
                                                          const float* __restrict__ q, int n,
                                                          int nmax, double3 L, double pi2_a2,
                                                          double fscale,
                                                          const double2* __restrict__ S,
                                                          float* __restrict__ force) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int w = 2 * nmax + 1;
  double ax = 0.0, ay = 0.0, az = 0.0;
  int h = 0;
  for (int n1 = 0; n1 <= nmax; ++n1) {
    const double2 e1 = tab[(size_t)(0 * w + n1 + nmax) * n + i];
    for (int n2 = n1 == 0 ? 0 : -nmax; n2 <= nmax; ++n2) {
      const double2 e12 = cmul(e1, tab[(size_t)(1 * w + n2 + nmax) * n + i]);
      for (int n3 = (n1 == 0 && n2 == 0) ? 1 : -nmax; n3 <= nmax; ++n3, ++h) {
        const double2 e = cmul(e12, tab[(size_t)(2 * w + n3 + nmax) * n + i]);
        const double2 s = S[h];
        const double mx = n1 / L.x, my = n2 / L.y, mz = n3 / L.z;
        const double m2 = mx * mx + my * my + mz * mz;
        const double t = (s.x * e.y - s.y * e.x) * exp(-pi2_a2 * m2) / m2;
        ax += t * mx;
        ay += t * my;
        az += t * mz;
      }
    }
  }
  // both m and -m: twice the half sum
  const double c = 2.0 * fscale * (double)q[i];
  force[i] += (float)(c * ax);
  force[n + i] += (float)(c * ay);
  force[2 * n + i] += (float)(c * az);
}

__global__ void __launch_bounds__(kEwThreads) k_ew_energy(const double* __restrict__ eterm, int K,
                                                          double escale, double* __restrict__ out) {
  __shared__ double s[kEwThreads];
  double acc = 0.0;
  for (int h = threadIdx.x; h < K; h += blockDim.x) acc += eterm[h];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = escale * 2.0 * s[0];   // both m and -m
}

// ---- fixed scratch for callers that cannot allocate --------------------
// One array per device (each GPU the library runs on holds its own copy until
// the process ends). Host code never passes `scratch` itself to a kernel: the
// name stands for a host-side shadow; the device address comes from
// hipGetSymbolAddress, taken once per device by ewald_scratch_setup.
static __device__ __align__(256) unsigned char scratch[kEwScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t ewald_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  // called with `device` current; a second call on a device keeps the first address
  if (__atomic_load_n(&g_scratch_ptr[device], __ATOMIC_ACQUIRE)) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  __atomic_store_n(&g_scratch_ptr[device], ptr, __ATOMIC_RELEASE);
  return hipSuccess;
}

size_t ewald_scratch_bytes(int n, int nmax, size_t* off_S, size_t* off_e) {
  const size_t w = 2 * (size_t)nmax + 1, K = (w * w * w - 1) / 2;
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t tab = up(3 * w * (size_t)n * sizeof(double2));
  const size_t S = up(K * sizeof(double2));
  if (off_S) *off_S = tab;
  if (off_e) *off_e = tab + S;
  return tab + S + up(K * sizeof(double));
}

hipError_t launch_ewald_direct_static(Ctx& c, const float* pos, float* force, double* energy,
                                      int nmax) {
  if (c.device < 0 || c.device >= kMaxDevices) return hipErrorInvalidDevice;
  unsigned char* base =
      static_cast<unsigned char*>(__atomic_load_n(&g_scratch_ptr[c.device], __ATOMIC_ACQUIRE));
  if (!base) return hipErrorNotInitialized;
  size_t off_S = 0, off_e = 0;
  if (ewald_scratch_bytes(c.n, nmax, &off_S, &off_e) > kEwScratchBytes)
    return hipErrorInvalidValue;
  return launch_ewald_direct(c, pos, force, energy, nmax, reinterpret_cast<double2*>(base),
                             reinterpret_cast<double2*>(base + off_S),
                             reinterpret_cast<double*>(base + off_e));
}

hipError_t launch_ewald_direct(Ctx& c, const float* pos, float* force, double* energy, int nmax,
                               double2* tab, double2* S, double* eterm) {
  const int n = c.n;
  const int w = 2 * nmax + 1;
  const int K = (w * w * w - 1) / 2;
  const double3 L = make_double3(c.box[0], c.box[1], c.box[2]);
  const double V = L.x * L.y * L.z;
  const double pi2_a2 = M_PI * M_PI / (c.alpha * c.alpha);
  k_ew_tables<<<(3 * n + 255) / 256, 256, 0, c.stream>>>(pos, n, L, nmax, tab);
  k_ew_structure<<<K, kEwThreads, 0, c.stream>>>(tab, c.q, n, nmax, L, pi2_a2, S, eterm);
  k_ew_forces<<<(n + kEwThreads - 1) / kEwThreads, kEwThreads, 0, c.stream>>>(
      tab, c.q, n, nmax, L, pi2_a2, 2.0 * c.coulomb_k / V, S, force);
  if (energy)
    k_ew_energy<<<1, kEwThreads, 0, c.stream>>>(eterm, K, c.coulomb_k / (2.0 * M_PI * V), energy);
  return hipGetLastError();
}

}  // namespace mdx
