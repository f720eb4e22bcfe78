// Observed data by bilinear finite elements on a uniform grid.
//
// The paper inverts data computed by a finer, conventional finite element
// model rather than by the scaled boundary discretisation itself (Section
// "Numerical examples"), which keeps the inversion free of the inverse crime.
// This file generates such data on the GPU: the scalar wave equation
// rho u_tt = div(rho c^2 grad u) + f with a free outer boundary, bilinear
// rectangles with one density per element, lumped (row-sum) mass and explicit
// central differences, M (u_{k+1} - 2 u_k + u_{k-1}) / dt^2 + K u_k = f_k.
//
// K is never assembled.  Each node applies the nine-point stencil that the
// four rectangles around it contribute: with A = hy / (6 hx), B = hx / (6 hy)
// and kappa = rho c^2 of each element, an element adds kappa times
//   (2A + 2B) to the node itself, (B - 2A) to its x-neighbour inside the
//   element, (A - 2B) to its y-neighbour, -(A + B) to the opposite corner,
// which is the element stiffness of bilinear shape functions on an hx x hy
// rectangle.  Elements outside the grid carry kappa = 0 (a zero border in the
// padded kappa array), which gives the free boundary without branches.
//
// Layout: u[shot][node], node (i, j) = j (nx + 1) + i, rows along x, so the
// x-neighbours of a wavefront's nodes are contiguous and the y-neighbours are
// the rows above and below.  One thread per (node, shot); blocks are spread
// so that consecutive node ranges sit on the same XCD (their halo rows then
// hit the same L2).
#include "sbfwi_internal.h"

#include <cmath>
#include <mutex>
#include <vector>

namespace {

constexpr int kFemBlock = 256;
constexpr int kXcds = 8;
constexpr int kMaxShots = 64;

struct FemDev {
  int nx, ny;
  int64_t nn;        // nodes
  double A, B;       // hy / (6 hx), hx / (6 hy)
  const double* kpad;   // [ny + 2][nx + 2], kappa of element (ie, je) at (je + 1, ie + 1)
  const double* minv;   // [nn] dt^2 / lumped mass
};

// kappa = rho c^2 into the padded array (zero border) and a status flag for
// densities that are not positive and finite.
__global__ void fem_kappa_kernel(int nx, int ny, const double* __restrict__ rho, double c2,
                                 double* __restrict__ kpad, int* status) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = (int64_t)(nx + 2) * (ny + 2);
  if (t >= total) return;
  int pj = (int)(t / (nx + 2)), pi = (int)(t - (int64_t)pj * (nx + 2));
  double k = 0.0;
  if (pi >= 1 && pi <= nx && pj >= 1 && pj <= ny) {
    double r = rho[(int64_t)(pj - 1) * nx + (pi - 1)];
    if (!(r > 0.0) || !isfinite(r)) *status = 1;
    k = r * c2;
  }
  kpad[t] = k;
}

// dt^2 / m at every node, m = sum over the (up to four) adjacent elements of
// rho_e hx hy / 4.
__global__ void fem_mass_kernel(int nx, int ny, const double* __restrict__ rho, double quarter_area,
                                double dt2, double* __restrict__ minv) {
  int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t nn = (int64_t)(nx + 1) * (ny + 1);
  if (node >= nn) return;
  int j = (int)(node / (nx + 1)), i = (int)(node - (int64_t)j * (nx + 1));
  double m = 0.0;
  for (int dj = -1; dj <= 0; ++dj)
    for (int di = -1; di <= 0; ++di) {
      int ie = i + di, je = j + dj;
      if (ie >= 0 && ie < nx && je >= 0 && je < ny) m += rho[(int64_t)je * nx + ie];
    }
  minv[node] = dt2 / (m * quarter_area);
}

__global__ void fem_zero_kernel(double* __restrict__ p, int64_t n) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = 0.0;
}

// traces[(s * n_rec + r) * n_steps + col] = u[s][rec[r]] for the shot of this
// block row; called by the first block of the row only.
__device__ inline void record(const double* __restrict__ us, const int64_t* __restrict__ rec, int n_rec,
                              double* __restrict__ traces, int s, int64_t n_steps, int64_t col) {
  for (int r = threadIdx.x; r < n_rec; r += blockDim.x)
    traces[((int64_t)s * n_rec + r) * n_steps + col] = us[rec[r]];
}

// One central-difference step for every (node, shot): reads u_k and u_{k-1}
// (in place in up), writes u_{k+1} into up.  Block 0 of each shot row also
// records u_k at the receivers (trace column k - 1).
__global__ __launch_bounds__(kFemBlock) void fem_step_kernel(FemDev g, const double* __restrict__ u,
                                                             double* __restrict__ up,
                                                             const int64_t* __restrict__ src,
                                                             const double* __restrict__ wavelet, int64_t n_steps,
                                                             int64_t k, const int64_t* __restrict__ rec, int n_rec,
                                                             double* __restrict__ traces) {
  const int s = blockIdx.y;
  const double* us = u + (int64_t)s * g.nn;
  // blocks b, b + 8, b + 16, ... land on one XCD: give them consecutive ranges
  const int per = gridDim.x / kXcds;
  const int lb = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
  if (lb == 0) record(us, rec, n_rec, traces, s, n_steps, k - 1);
  const int64_t node = (int64_t)lb * kFemBlock + threadIdx.x;
  if (node >= g.nn) return;
  const int w = g.nx + 1;
  const int j = (int)(node / w), i = (int)(node - (int64_t)j * w);
  const double* kp = g.kpad + (int64_t)j * (g.nx + 2) + i;
  const double kSW = kp[0], kSE = kp[1], kNW = kp[g.nx + 2], kNE = kp[g.nx + 3];
  const int im = i > 0 ? i - 1 : 0, ip = i < g.nx ? i + 1 : g.nx;
  const int64_t r0 = (int64_t)(j > 0 ? j - 1 : 0) * w, r1 = (int64_t)j * w, r2 = (int64_t)(j < g.ny ? j + 1 : g.ny) * w;
  const double uc = us[r1 + i];
  const double ku = (2.0 * g.A + 2.0 * g.B) * ((kNE + kNW) + (kSE + kSW)) * uc
                  + (g.B - 2.0 * g.A) * ((kNE + kSE) * us[r1 + ip] + (kNW + kSW) * us[r1 + im])
                  + (g.A - 2.0 * g.B) * ((kNE + kNW) * us[r2 + i] + (kSE + kSW) * us[r0 + i])
                  - (g.A + g.B) * ((kNE * us[r2 + ip] + kNW * us[r2 + im]) + (kSE * us[r0 + ip] + kSW * us[r0 + im]));
  const double f = node == src[s] ? wavelet[(int64_t)s * n_steps + (k - 1)] : 0.0;
  double* ps = up + (int64_t)s * g.nn;
  ps[node] = 2.0 * uc - ps[node] + g.minv[node] * (f - ku);
}

__global__ void fem_record_kernel(const double* __restrict__ u, int64_t nn, const int64_t* __restrict__ rec,
                                  int n_rec, double* __restrict__ traces, int64_t n_steps, int64_t col) {
  record(u + (int64_t)blockIdx.x * nn, rec, n_rec, traces, blockIdx.x, n_steps, col);
}

// Node ids checked on the device: status bit 2 for an id outside [0, nn).
__global__ void fem_check_nodes_kernel(const int64_t* __restrict__ nodes, int count, int64_t nn, int* status) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count && (nodes[t] < 0 || nodes[t] >= nn)) atomicOr(status, 2);
}

__global__ void fem_clear_status_kernel(int* status) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *status = 0;
}

// Device work buffers of one call: padded kappa, dt^2 / m, the two wavefields.
struct FemWork {
  double *kpad = nullptr, *minv = nullptr, *u0 = nullptr, *u1 = nullptr;
  int* status = nullptr;
};

// Coefficients, zero initial fields and the time loop (buffers in w); the
// densities are checked through w.status, which the caller has cleared.
int fem_run(int nx, int ny, double hx, double hy, const double* rho_elem, double c, double dt, int n_shots,
            int64_t n_steps, const int64_t* src_node, const double* wavelet, int n_rec, const int64_t* rec_node,
            double* traces, const FemWork& w, int check_bits, hipStream_t s) {
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1);
  const int64_t npad = (int64_t)(nx + 2) * (ny + 2);
  auto blocks = [](int64_t n) { return (unsigned)((n + kFemBlock - 1) / kFemBlock); };
  fem_kappa_kernel<<<blocks(npad), kFemBlock, 0, s>>>(nx, ny, rho_elem, c * c, w.kpad, w.status);
  fem_mass_kernel<<<blocks(nn), kFemBlock, 0, s>>>(nx, ny, rho_elem, hx * hy / 4.0, dt * dt, w.minv);
  fem_zero_kernel<<<blocks(nn * n_shots), kFemBlock, 0, s>>>(w.u0, nn * n_shots);
  fem_zero_kernel<<<blocks(nn * n_shots), kFemBlock, 0, s>>>(w.u1, nn * n_shots);
  SBFWI_HIP(hipGetLastError());
  int status = 0;
  SBFWI_HIP(hipMemcpyAsync(&status, w.status, sizeof(int), hipMemcpyDeviceToHost, s));
  SBFWI_HIP(hipStreamSynchronize(s));
  if ((status & 2) && (check_bits & 2)) return sbfwi_fail(SBFWI_EINVAL, "a source or receiver node is out of range");
  if (status & 1) return sbfwi_fail(SBFWI_EINVAL, "element densities must be positive and finite");

  FemDev g{nx, ny, nn, hy / (6.0 * hx), hx / (6.0 * hy), w.kpad, w.minv};
  // grid padded to a multiple of the XCD count so the block spread is a bijection
  const unsigned nb = (blocks(nn) + kXcds - 1) / kXcds * kXcds;
  double* u = w.u1;   // u_k   (k = 1: zero)
  double* up = w.u0;  // u_{k-1}, overwritten with u_{k+1}
  for (int64_t k = 1; k < n_steps; ++k) {
    {
      ProfScope ps(PK_FEM_STEP, s);
      fem_step_kernel<<<dim3(nb, n_shots), kFemBlock, 0, s>>>(g, u, up, src_node, wavelet, n_steps, k, rec_node,
                                                              n_rec, traces);
    }
    double* t = u;
    u = up;
    up = t;
  }
  if (n_rec > 0) fem_record_kernel<<<n_shots, kFemBlock, 0, s>>>(u, nn, rec_node, n_rec, traces, n_steps, n_steps - 1);
  SBFWI_HIP(hipGetLastError());
  SBFWI_HIP(hipStreamSynchronize(s));
  return SBFWI_OK;
}

// Argument checks shared by both entry points (host values only).
int fem_check_args(int nx, int ny, double lx, double ly, const double* rho_elem, double c, double dt, int n_shots,
                   int64_t n_steps, const int64_t* src_node, const double* wavelet, int n_rec,
                   const int64_t* rec_node, double* traces) {
  if (nx < 1 || ny < 1 || nx > 32768 || ny > 32768) return sbfwi_fail(SBFWI_EINVAL, "nx, ny must be in 1..32768");
  if (!(lx > 0.0) || !(ly > 0.0) || !std::isfinite(lx) || !std::isfinite(ly))
    return sbfwi_fail(SBFWI_EINVAL, "lx, ly must be positive");
  if (!(c > 0.0) || !(dt > 0.0) || !std::isfinite(c) || !std::isfinite(dt))
    return sbfwi_fail(SBFWI_EINVAL, "c and dt must be positive");
  if (n_shots < 1 || n_shots > kMaxShots) return sbfwi_fail(SBFWI_EINVAL, "n_shots must be in 1..%d", kMaxShots);
  if (n_steps < 1) return sbfwi_fail(SBFWI_EINVAL, "n_steps must be positive");
  if (n_rec < 0 || (n_rec > 0 && (!rec_node || !traces))) return sbfwi_fail(SBFWI_EINVAL, "bad receivers");
  if (!rho_elem || !src_node || !wavelet) return sbfwi_fail(SBFWI_EINVAL, "NULL argument");
  const double hx = lx / nx, hy = ly / ny;
  // central differences are stable for dt^2 lambda_max(M^-1 K) <= 4; the row
  // sums bound lambda_max by 4 c^2 (1/hx^2 + 1/hy^2)
  if (dt * c * std::sqrt(1.0 / (hx * hx) + 1.0 / (hy * hy)) > 1.0)
    return sbfwi_fail(SBFWI_EINVAL, "dt = %g exceeds the stable step %g of the grid", dt,
                      1.0 / (c * std::sqrt(1.0 / (hx * hx) + 1.0 / (hy * hy))));
  return SBFWI_OK;
}

// Work buffers of one call; released after the stream has drained (also on
// error returns after launches).
struct FemBuffers {
  hipStream_t s = nullptr;
  double *kpad = nullptr, *minv = nullptr, *u0 = nullptr, *u1 = nullptr;
  int* status = nullptr;
  ~FemBuffers() {
    (void)hipStreamSynchronize(s);
    sbfwi_dev_free(kpad);
    sbfwi_dev_free(minv);
    sbfwi_dev_free(u0);
    sbfwi_dev_free(u1);
    sbfwi_dev_free(status);
  }
};

int check_nodes(const int64_t* dev, int count, int64_t nn, hipStream_t s, const char* what) {
  std::vector<int64_t> h(count);
  SBFWI_HIP(hipMemcpyAsync(h.data(), dev, count * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SBFWI_HIP(hipStreamSynchronize(s));
  for (int64_t v : h)
    if (v < 0 || v >= nn) return sbfwi_fail(SBFWI_EINVAL, "%s node %lld out of range", what, (long long)v);
  return SBFWI_OK;
}

}  // namespace

extern "C" int sbfwi_fem_forward(int nx, int ny, double lx, double ly, const double* rho_elem, double c,
                                 double dt, int n_shots, int64_t n_steps, const int64_t* src_node,
                                 const double* wavelet, int n_rec, const int64_t* rec_node, double* traces,
                                 hipStream_t s) {
  SBFWI_CHECK(fem_check_args(nx, ny, lx, ly, rho_elem, c, dt, n_shots, n_steps, src_node, wavelet, n_rec,
                             rec_node, traces));
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1);
  SBFWI_CHECK(check_nodes(src_node, n_shots, nn, s, "source"));
  if (n_rec > 0) SBFWI_CHECK(check_nodes(rec_node, n_rec, nn, s, "receiver"));

  FemBuffers b;
  b.s = s;
  const int64_t npad = (int64_t)(nx + 2) * (ny + 2);
  SBFWI_CHECK(sbfwi_alloc(&b.kpad, npad));
  SBFWI_CHECK(sbfwi_alloc(&b.minv, nn));
  SBFWI_CHECK(sbfwi_alloc(&b.u0, nn * n_shots));
  SBFWI_CHECK(sbfwi_alloc(&b.u1, nn * n_shots));
  SBFWI_CHECK(sbfwi_alloc(&b.status, 1));
  SBFWI_HIP(hipMemsetAsync(b.status, 0, sizeof(int), s));
  FemWork w{b.kpad, b.minv, b.u0, b.u1, b.status};
  return fem_run(nx, ny, lx / nx, ly / ny, rho_elem, c, dt, n_shots, n_steps, src_node, wavelet, n_rec, rec_node,
                 traces, w, 0, s);
}

// ---------------------------------------------------------------------------
// Allocation-free variant: the work buffers live in scratch, a static device
// array that every GPU the library runs on holds until the process ends.  Its
// device address is taken once per device (hipGetSymbolAddress, with that
// device current) and kept; host code uses only that address, never the
// array's name.  Every call on a GPU shares the array: calls that overlap on
// one GPU race.  Layout: the status word, then kpad, minv, u0, u1, each at a
// 256-byte boundary; everything that must start at zero is cleared by kernels.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kFemScratchBytes = (size_t)48 << 20;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) double scratch[kFemScratchBytes / sizeof(double)];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of scratch on the current device (taken on its first use there).
int scratch_address(void** out) {
  int dev = -1;
  SBFWI_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return sbfwi_fail(SBFWI_EINVAL, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return sbfwi_fail(SBFWI_EHIP, "hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SBFWI_OK;
}

inline size_t round256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

extern "C" int sbfwi_fem_forward_noalloc(int nx, int ny, double lx, double ly, const double* rho_elem, double c,
                                         double dt, int n_shots, int64_t n_steps, const int64_t* src_node,
                                         const double* wavelet, int n_rec, const int64_t* rec_node,
                                         double* traces, hipStream_t s) {
  SBFWI_CHECK(fem_check_args(nx, ny, lx, ly, rho_elem, c, dt, n_shots, n_steps, src_node, wavelet, n_rec,
                             rec_node, traces));
  const int64_t nn = (int64_t)(nx + 1) * (ny + 1);
  const int64_t npad = (int64_t)(nx + 2) * (ny + 2);
  const size_t o_kpad = 256;
  const size_t o_minv = o_kpad + round256(sizeof(double) * npad);
  const size_t o_u0 = o_minv + round256(sizeof(double) * nn);
  const size_t o_u1 = o_u0 + round256(sizeof(double) * nn * n_shots);
  const size_t need = o_u1 + round256(sizeof(double) * nn * n_shots);
  if (need > kFemScratchBytes)
    return sbfwi_fail(SBFWI_EINVAL,
                      "grid %d x %d with %d shots needs %zu bytes of scratch; the allocation-free call has %zu",
                      nx, ny, n_shots, need, kFemScratchBytes);
  void* base = nullptr;
  SBFWI_CHECK(scratch_address(&base));
  char* b = static_cast<char*>(base);
  FemWork w;
  w.status = reinterpret_cast<int*>(b);
  w.kpad = reinterpret_cast<double*>(b + o_kpad);
  w.minv = reinterpret_cast<double*>(b + o_minv);
  w.u0 = reinterpret_cast<double*>(b + o_u0);
  w.u1 = reinterpret_cast<double*>(b + o_u1);
  // the array keeps the last call's contents: the status word is cleared here,
  // the wavefields by fem_run; node ids are checked on the device
  fem_clear_status_kernel<<<1, 64, 0, s>>>(w.status);
  fem_check_nodes_kernel<<<(n_shots + 255) / 256, 256, 0, s>>>(src_node, n_shots, nn, w.status);
  if (n_rec > 0) fem_check_nodes_kernel<<<(n_rec + 255) / 256, 256, 0, s>>>(rec_node, n_rec, nn, w.status);
  SBFWI_HIP(hipGetLastError());
  return fem_run(nx, ny, lx / nx, ly / ny, rho_elem, c, dt, n_shots, n_steps, src_node, wavelet, n_rec, rec_node,
                 traces, w, 2, s);
}
