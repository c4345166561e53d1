// div B cleaning in Fourier space (Section 3, eq. clean1, eq. clean2) for
// periodic boxes: the potential phi solves the staggered Laplacian
// ddxup(ddxdn(phi)) + ddyup(ddydn(phi)) + ddzup(ddzdn(phi)) = div B, with
// div B = ddxup(B_x) + ddyup(B_y) + ddzup(B_z) at the centres; on a Fourier
// mode the Laplacian is multiplication by -(K_x^2 + K_y^2 + K_z^2), K the
// sixth-order derivative symbol, zero only for the mean mode (whose phi is
// 0).  Then B_a -= ddadn(phi) on the faces, which leaves a discretely
// solenoidal field.  The transforms are rocFFT real-to-complex and back.
#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <cmath>
#include <mutex>

#include "mhd_clean.hpp"
#include "mhd_zmarch.hpp"

namespace smhd {

namespace {

constexpr int kCleanBlock = 256;

// Cell coordinates of box-local index q in 32-bit arithmetic (boxes hold
// fewer than 2^31 cells; 64-bit division is emulated and slow).
__device__ __forceinline__ void clean_coords(unsigned q, unsigned nx, unsigned ny, int& i, int& j, int& k) {
  const unsigned qx = q / nx, qy = qx / ny;
  i = (int)(q - qx * nx);
  j = (int)(qx - qy * ny);
  k = (int)qy;
}

// The stencil kernels march along z: one thread per (x, y) column and
// chunk of kCleanZ planes, the z operand in a register window of six
// planes, so each plane of it is read once per chunk (plus the window's
// warm-up) instead of six times.  A workgroup covers kCleanTX x kCleanTY
// columns, so the rows of a y stencil are mostly shared within it.
constexpr int kCleanZ = 32;
constexpr int kCleanTX = 64, kCleanTY = kCleanBlock / kCleanTX;

__device__ __forceinline__ int wrapz(int k, int n) { return k < 0 ? k + n : (k >= n ? k - n : k); }

// div B at the centres of one box (box-local output index).
template <class T>
__global__ __launch_bounds__(kCleanBlock) void k_clean_div(BoxDev b, const T* __restrict__ bx,
                                                           const T* __restrict__ by,
                                                           const T* __restrict__ bz, T* __restrict__ div) {
  const int i = (int)(blockIdx.x * kCleanTX + threadIdx.x % kCleanTX);
  const int j = (int)(blockIdx.y * kCleanTY + threadIdx.x / kCleanTX);
  if (i >= b.nx || j >= b.ny) return;
  const unsigned nxy = (unsigned)b.nx * (unsigned)b.ny;
  const unsigned q = (unsigned)j * (unsigned)b.nx + (unsigned)i;
  const int z0 = (int)blockIdx.z * kCleanZ, z1 = min(z0 + kCleanZ, b.nzt);
  const Geo<T> g(b);
  // window of bz at planes k-2 .. k+3 (the up derivative's samples)
  T w[6];
#pragma unroll
  for (int m = 0; m < 5; ++m) w[m] = bz[g.at(i, j, wrapz(z0 - 2 + m, b.nzt))];
  for (int k = z0; k < z1; ++k) {
    w[5] = bz[g.at(i, j, wrapz(k + 3, b.nzt))];
    div[(long long)k * nxy + q] = op6<1, 1, T>([&](int m) { return bx[g.at(i + m, j, k)]; }, g.hxi) +
                                  op6<1, 1, T>([&](int m) { return by[g.at(i, j + m, k)]; }, g.hyi) +
                                  op6<1, 1, T>([&](int m) { return w[m + 2]; }, g.hzi);
#pragma unroll
    for (int m = 0; m < 5; ++m) w[m] = w[m + 1];
  }
}

// phi^ = -div^ / (K_x^2 + K_y^2 + K_z^2) times `scale` (the 1/N of the
// unnormalised inverse transform); the mean mode's phi is 0.  F holds
// (nx/2 + 1) x ny x nz complex values, x fastest.
template <class T, class C>
__global__ __launch_bounds__(kCleanBlock) void k_clean_solve(C* __restrict__ F, const T* __restrict__ k2x,
                                                             const T* __restrict__ k2y,
                                                             const T* __restrict__ k2z, int nxh, int ny, int nz,
                                                             T scale) {
  const unsigned q = blockIdx.x * kCleanBlock + threadIdx.x;
  if ((long long)q >= (long long)nxh * ny * nz) return;
  int i, j, k;
  clean_coords(q, (unsigned)nxh, (unsigned)ny, i, j, k);
  const T L = k2x[i] + k2y[j] + k2z[k];
  C v = F[q];
  const T s = L > T(0) ? -scale / L : T(0);
  v.x *= s;
  v.y *= s;
  F[q] = v;
}

// B_a -= ddadn(phi) on the faces of one box (phi box-local).
template <class T>
__global__ __launch_bounds__(kCleanBlock) void k_clean_apply(BoxDev b, const T* __restrict__ phi,
                                                             T* __restrict__ bx, T* __restrict__ by,
                                                             T* __restrict__ bz) {
  const int i = (int)(blockIdx.x * kCleanTX + threadIdx.x % kCleanTX);
  const int j = (int)(blockIdx.y * kCleanTY + threadIdx.x / kCleanTX);
  if (i >= b.nx || j >= b.ny) return;
  const unsigned nxy = (unsigned)b.nx * (unsigned)b.ny;
  const unsigned q = (unsigned)j * (unsigned)b.nx + (unsigned)i;
  const int z0 = (int)blockIdx.z * kCleanZ, z1 = min(z0 + kCleanZ, b.nzt);
  const Geo<T> g(b);
  auto at = [&](int x, int y, int z) {
    x = x < 0 ? x + b.nx : (x >= b.nx ? x - b.nx : x);
    y = y < 0 ? y + b.ny : (y >= b.ny ? y - b.ny : y);
    return phi[(long long)z * nxy + (long long)y * b.nx + x];
  };
  // window of phi at planes k-3 .. k+2 (the down derivative's samples)
  T w[6];
#pragma unroll
  for (int m = 0; m < 5; ++m) w[m] = at(i, j, wrapz(z0 - 3 + m, b.nzt));
  for (int k = z0; k < z1; ++k) {
    w[5] = at(i, j, wrapz(k + 2, b.nzt));
    const long long o = b.off + (long long)k * nxy + q;
    bx[o] -= op6<1, 0, T>([&](int m) { return at(i + m, j, k); }, g.hxi);
    by[o] -= op6<1, 0, T>([&](int m) { return at(i, j + m, k); }, g.hyi);
    bz[o] -= op6<1, 0, T>([&](int m) { return w[m + 3]; }, g.hzi);
#pragma unroll
    for (int m = 0; m < 5; ++m) w[m] = w[m + 1];
  }
}

// K(theta_m)^2 of the sixth-order staggered derivative (eq. deriv) for
// modes m = 0..count-1 of a periodic axis of n cells and spacing h.
void symbol_sq(int n, int count, double h, std::vector<double>& out) {
  const double d[3] = {75.0 / 64.0, -25.0 / 384.0, 3.0 / 640.0};
  for (int m = 0; m < count; ++m) {
    const double th = 2.0 * M_PI * m / n;
    double K = 0.0;
    for (int p = 1; p <= 3; ++p) K += d[p - 1] * std::sin((2 * p - 1) * th / 2.0);
    K *= 2.0 / h;
    out.push_back(K * K);
  }
}

std::once_flag g_rocfft_once;
rocfft_status g_rocfft_setup = rocfft_status_success;

}  // namespace

struct CleanState {
  struct Plan {
    int nx, ny, nz;
    rocfft_plan fwd = nullptr, inv = nullptr;
  };
  std::vector<Plan> plans;
  int dtype = -1;
  void* real = nullptr;   // div B, then phi: the largest box's cells
  void* cplx = nullptr;   // its transform
  void* work = nullptr;   // rocFFT's work buffer, the largest the plans ask
  void* ktab = nullptr;   // K^2 per axis and box
  size_t work_bytes = 0;
  std::vector<long long> koff;   // per box: offset of its x, y, z tables in ktab
  rocfft_execution_info info = nullptr;
};

void clean_free(CleanState* s) {
  if (!s) return;
  for (auto& p : s->plans) {
    if (p.fwd) (void)rocfft_plan_destroy(p.fwd);
    if (p.inv) (void)rocfft_plan_destroy(p.inv);
  }
  if (s->info) (void)rocfft_execution_info_destroy(s->info);
  (void)hipFree(s->real);
  (void)hipFree(s->cplx);
  (void)hipFree(s->work);
  (void)hipFree(s->ktab);
  delete s;
}

template <class T>
int clean_boxes(CleanState** sp, const std::vector<BoxDev>& boxes, P8<T> f, hipStream_t stream,
                std::string& err) {
  using C = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
  const rocfft_precision prec = sizeof(T) == 4 ? rocfft_precision_single : rocfft_precision_double;
  std::call_once(g_rocfft_once, [] { g_rocfft_setup = rocfft_setup(); });
  if (g_rocfft_setup != rocfft_status_success) {
    err = "rocfft_setup failed";
    return 1;
  }
  if (!*sp) {
    CleanState* s = new CleanState;
    s->dtype = sizeof(T);
    // one plan pair per distinct box shape, buffers for the largest box
    long long ncell = 0, ncplx = 0;
    std::vector<double> k2;
    for (const BoxDev& b : boxes) {
      ncell = std::max(ncell, b.ncell);
      ncplx = std::max(ncplx, (long long)(b.nx / 2 + 1) * b.ny * b.nzt);
      s->koff.push_back((long long)k2.size());
      symbol_sq(b.nx, b.nx / 2 + 1, b.dx, k2);
      symbol_sq(b.ny, b.ny, b.dy, k2);
      symbol_sq(b.nzt, b.nzt, b.dz, k2);
      bool have = false;
      for (const auto& p : s->plans) have |= p.nx == b.nx && p.ny == b.ny && p.nz == b.nzt;
      if (have) continue;
      CleanState::Plan p;
      p.nx = b.nx;
      p.ny = b.ny;
      p.nz = b.nzt;
      const size_t len[3] = {(size_t)b.nx, (size_t)b.ny, (size_t)b.nzt};   // fastest first
      if (rocfft_plan_create(&p.fwd, rocfft_placement_notinplace, rocfft_transform_type_real_forward, prec, 3,
                             len, 1, nullptr) != rocfft_status_success ||
          rocfft_plan_create(&p.inv, rocfft_placement_notinplace, rocfft_transform_type_real_inverse, prec, 3,
                             len, 1, nullptr) != rocfft_status_success) {
        s->plans.push_back(p);
        clean_free(s);
        err = "rocfft_plan_create failed";
        return 1;
      }
      size_t w1 = 0, w2 = 0;
      (void)rocfft_plan_get_work_buffer_size(p.fwd, &w1);
      (void)rocfft_plan_get_work_buffer_size(p.inv, &w2);
      s->work_bytes = std::max(s->work_bytes, std::max(w1, w2));
      s->plans.push_back(p);
    }
    std::vector<T> kt(k2.begin(), k2.end());
    if (hipMalloc(&s->real, sizeof(T) * ncell) != hipSuccess ||
        hipMalloc(&s->cplx, sizeof(C) * ncplx) != hipSuccess ||
        (s->work_bytes && hipMalloc(&s->work, s->work_bytes) != hipSuccess) ||
        hipMalloc(&s->ktab, sizeof(T) * kt.size()) != hipSuccess ||
        hipMemcpy(s->ktab, kt.data(), sizeof(T) * kt.size(), hipMemcpyHostToDevice) != hipSuccess ||
        rocfft_execution_info_create(&s->info) != rocfft_status_success) {
      clean_free(s);
      err = "allocation failed";
      return 2;
    }
    *sp = s;
  }
  CleanState* s = *sp;
  if (rocfft_execution_info_set_stream(s->info, stream) != rocfft_status_success ||
      (s->work && rocfft_execution_info_set_work_buffer(s->info, s->work, s->work_bytes) != rocfft_status_success)) {
    err = "rocfft execution info";
    return 1;
  }
  T* real = static_cast<T*>(s->real);
  C* cplx = static_cast<C*>(s->cplx);
  const T* kt = static_cast<const T*>(s->ktab);
  for (size_t bi = 0; bi < boxes.size(); ++bi) {
    const BoxDev& b = boxes[bi];
    const CleanState::Plan* p = nullptr;
    for (const auto& q : s->plans)
      if (q.nx == b.nx && q.ny == b.ny && q.nz == b.nzt) p = &q;
    const int nxh = b.nx / 2 + 1;
    const dim3 gc((unsigned)((b.nx + kCleanTX - 1) / kCleanTX), (unsigned)((b.ny + kCleanTY - 1) / kCleanTY),
                  (unsigned)((b.nzt + kCleanZ - 1) / kCleanZ));
    const long long nc = (long long)nxh * b.ny * b.nzt;
    const dim3 gk((unsigned)((nc + kCleanBlock - 1) / kCleanBlock));
    hipLaunchKernelGGL(k_clean_div<T>, gc, dim3(kCleanBlock), 0, stream, b, f.p[5], f.p[6], f.p[7], real);
    void* in1[1] = {real};
    void* out1[1] = {cplx};
    if (rocfft_execute(p->fwd, in1, out1, s->info) != rocfft_status_success) {
      err = "rocfft forward transform failed";
      return 1;
    }
    const T* kx = kt + s->koff[bi];
    hipLaunchKernelGGL((k_clean_solve<T, C>), gk, dim3(kCleanBlock), 0, stream, cplx, kx, kx + nxh,
                       kx + nxh + b.ny, nxh, b.ny, b.nzt, T(1.0 / (double)b.ncell));
    void* in2[1] = {cplx};
    void* out2[1] = {real};
    if (rocfft_execute(p->inv, in2, out2, s->info) != rocfft_status_success) {
      err = "rocfft inverse transform failed";
      return 1;
    }
    hipLaunchKernelGGL(k_clean_apply<T>, gc, dim3(kCleanBlock), 0, stream, b, (const T*)real, f.p[5], f.p[6],
                       f.p[7]);
  }
  return 0;
}

template int clean_boxes<float>(CleanState**, const std::vector<BoxDev>&, P8<float>, hipStream_t, std::string&);
template int clean_boxes<double>(CleanState**, const std::vector<BoxDev>&, P8<double>, hipStream_t,
                                 std::string&);

}  // namespace smhd
