// Synthetic Hessian samplers (h2_sampler_fn compatible), standing in for the
// user's PDE solver: the method only ever sees products of the Hessian with
// blocks of vectors, each costing a forward and an adjoint solve (Sec. 2 and
// Sec. 3.3).  All operate on user-ordered column-major blocks.
//
//   kernel     H_ij = exp(-|p_i - p_j| / ell) + shift delta_ij, evaluated on the
//              fly in 64 x 64 tiles (no N^2 storage)
//   diffusion  Gauss-Newton Hessian of an initial-condition inversion for
//              explicit-Euler heat flow, F^T F / sigma^2 + gamma (I - beta Lap)^2;
//              one workgroup per column keeps the whole grid in LDS for all
//              forward and adjoint steps
//   advdiff    misfit Gauss-Newton Hessian of first-order upwind
//              advection-diffusion with bilinear point observations
#include <algorithm>
#include <cmath>
#include <functional>
#include <type_traits>
#include <vector>

#include "internal.h"
#include "kernels_common.h"

namespace h2 {

h2_status guarded_status(const std::function<void()>& f);

// ------------------------------------------------------------------ kernel matrix
struct KernelCtx {
  int kind = 1;
  int n, dim;
  double ell, shift;
  DevBuf pts;  // n x 3 (zero padded), user order
};

constexpr int KT = 64;   // tile of rows / columns of H
constexpr int KC = 16;   // vectors per block

// rows r0 .. r0 + KT - 1 and columns c0 .. c0 + KC - 1 of y = H om for one
// kernel matrix (points P, n x 3): the whole of one workgroup's work
__device__ __forceinline__ void kernel_tile(int r0, int c0, int n, int ncols,
                                            const double* __restrict__ P, double inv_ell,
                                            double shift, const double* __restrict__ om, int ldo,
                                            double* __restrict__ y, int ldy) {
  __shared__ double Ht[KT][KT + 1];
  __shared__ double Ot[KT][KC];
  __shared__ double pr[KT][3];
  const int nc = min(KC, ncols - c0);
  const int tid = threadIdx.x;
  for (int e = tid; e < KT * 3; e += 256) {
    const int i = e / 3, d = e % 3;
    pr[i][d] = (r0 + i < n) ? P[(size_t)(r0 + i) * 3 + d] : 0.0;
  }
  // each thread: row i = tid / 4, columns j = (tid % 4) * 4 .. +3
  const int ri = tid >> 2, cj = (tid & 3) * 4;
  double acc[4] = {0, 0, 0, 0};
  for (int s0 = 0; s0 < n; s0 += KT) {
    __syncthreads();
    for (int e = tid; e < KT * KT; e += 256) {
      const int i = e / KT, j = e % KT;
      const int gj = s0 + j;
      double h = 0;
      if (r0 + i < n && gj < n) {
        const double dx = pr[i][0] - P[(size_t)gj * 3 + 0];
        const double dy = pr[i][1] - P[(size_t)gj * 3 + 1];
        const double dz = pr[i][2] - P[(size_t)gj * 3 + 2];
        h = exp(-sqrt(dx * dx + dy * dy + dz * dz) * inv_ell);
        if (r0 + i == gj) h += shift;
      }
      Ht[i][j] = h;
    }
    for (int e = tid; e < KT * KC; e += 256) {
      const int j = e / KC, v = e % KC;
      Ot[j][v] = (s0 + j < n && v < nc) ? om[(size_t)(c0 + v) * ldo + s0 + j] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int j = 0; j < KT; ++j) {
      const double h = Ht[ri][j];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = fma(h, Ot[j][cj + q], acc[q]);
    }
  }
  if (r0 + ri < n)
    for (int q = 0; q < 4; ++q)
      if (cj + q < nc) y[(size_t)(c0 + cj + q) * ldy + r0 + ri] = acc[q];
}

__global__ __launch_bounds__(256) void k_kernel_apply(int n, int ncols, const double* __restrict__ P,
                                                      double inv_ell, double shift,
                                                      const double* __restrict__ om, int ldo,
                                                      double* __restrict__ y, int ldy) {
  kernel_tile(blockIdx.x * KT, blockIdx.y * KC, n, ncols, P, inv_ell, shift, om, ldo, y, ldy);
}

// Several kernel matrices in one launch over the packed layout (problem i
// owns rows off[i] .. off[i+1] - 1 of om, y and P): one workgroup per row
// tile of one problem; each tile is computed exactly as k_kernel_apply does
struct KernelBatchCtx {
  int kind = 5;
  int nprob;
  std::vector<int64_t> off;
  DevBuf pts, tiles, prm;  // points (rows x 3); tile -> (problem, r0); (1/ell, shift) per problem
  DevBuf tiles_off;        // row offsets (nprob + 1) on the device
  int ntiles;
};

__global__ __launch_bounds__(256) void k_kernel_apply_batched(
    const int32_t* __restrict__ tiles, const int64_t* __restrict__ off,
    const double* __restrict__ prm, const double* __restrict__ P, int ncols,
    const double* __restrict__ om, int ld, double* __restrict__ y) {
  const int i = tiles[2 * blockIdx.x], r0 = tiles[2 * blockIdx.x + 1];
  const int64_t o = off[i];
  const int n = (int)(off[i + 1] - o);
  kernel_tile(r0, blockIdx.y * KC, n, ncols, P + (size_t)o * 3, prm[2 * i], prm[2 * i + 1],
              om + o, ld, y + o, ld);
}

// ------------------------------------------------------------------ explicit stepping
struct StepCtx {
  int kind = 2;      // 2 diffusion, 3 advdiff
  int g, steps;
  std::vector<int> obs_steps;      // sorted step numbers
  double sigma;
  // diffusion
  double cdiff = 0;                // dt * kappa / h^2
  double gamma = 0, beta_h2 = 0;   // gamma, beta / h^2
  DevBuf obs_idx;                  // node indices of the observation points
  int nobs = 0;
  // advdiff: per-node stencil coefficients (centre, west, east, south, north)
  DevBuf coef;
  DevBuf bil_idx, bil_w;           // 4 nodes and weights per observation (-1: none)
  DevBuf obs_step_flag;            // steps + 1 ints: observation slot or -1
  DevBuf work;                     // per-call observation storage
};

// one block per column; the grid lives in LDS; PPT points per thread
template <int PPT>
__global__ __launch_bounds__(256) void k_diffusion_apply(
    int g, int steps, double cdiff, double inv_sig2, double gamma, double bh2,
    const int32_t* __restrict__ oidx, int nobs, const int32_t* __restrict__ slot,
    int nslots, const double* __restrict__ om, int ldo, double* __restrict__ y, int ldy,
    double* __restrict__ obs_store) {
  extern __shared__ double u[];
  const int N = g * g;
  const int col = blockIdx.x;
  const int tid = threadIdx.x;
  const double* v = om + (size_t)col * ldo;
  double* ob = obs_store + (size_t)col * nslots * nobs;
  double nv[PPT];
  for (int q = 0; q < PPT; ++q) {
    const int i = tid + 256 * q;
    if (i < N) u[i] = v[i];
  }
  __syncthreads();
  auto lap_at = [&](int i) {
    const int ix = i % g, iy = i / g;
    double s = -4.0 * u[i];
    if (ix > 0) s += u[i - 1];
    if (ix < g - 1) s += u[i + 1];
    if (iy > 0) s += u[i - g];
    if (iy < g - 1) s += u[i + g];
    return s;
  };
  // forward steps with observations
  for (int s = 1; s <= steps; ++s) {
    for (int q = 0; q < PPT; ++q) {
      const int i = tid + 256 * q;
      if (i < N) nv[q] = u[i] + cdiff * lap_at(i);
    }
    __syncthreads();
    for (int q = 0; q < PPT; ++q) {
      const int i = tid + 256 * q;
      if (i < N) u[i] = nv[q];
    }
    __syncthreads();
    const int sl = slot[s];
    if (sl >= 0)
      for (int o = tid; o < nobs; o += 256) ob[sl * nobs + o] = u[oidx[o]];
    __syncthreads();
  }
  // adjoint steps (the step operator is symmetric)
  for (int q = 0; q < PPT; ++q) {
    const int i = tid + 256 * q;
    if (i < N) u[i] = 0.0;
  }
  __syncthreads();
  for (int s = steps; s >= 1; --s) {
    const int sl = slot[s];
    if (sl >= 0)
      for (int o = tid; o < nobs; o += 256) u[oidx[o]] += ob[sl * nobs + o];
    __syncthreads();
    for (int q = 0; q < PPT; ++q) {
      const int i = tid + 256 * q;
      if (i < N) nv[q] = u[i] + cdiff * lap_at(i);
    }
    __syncthreads();
    for (int q = 0; q < PPT; ++q) {
      const int i = tid + 256 * q;
      if (i < N) u[i] = nv[q];
    }
    __syncthreads();
  }
  // misfit part
  double mis[PPT];
  for (int q = 0; q < PPT; ++q) {
    const int i = tid + 256 * q;
    mis[q] = i < N ? u[i] * inv_sig2 : 0.0;
  }
  __syncthreads();
  // regularisation gamma (I - beta Lap)^2 v
  for (int q = 0; q < PPT; ++q) {
    const int i = tid + 256 * q;
    if (i < N) u[i] = v[i];
  }
  __syncthreads();
  for (int rep = 0; rep < 2; ++rep) {
    for (int q = 0; q < PPT; ++q) {
      const int i = tid + 256 * q;
      if (i < N) nv[q] = u[i] - bh2 * lap_at(i);
    }
    __syncthreads();
    for (int q = 0; q < PPT; ++q) {
      const int i = tid + 256 * q;
      if (i < N) u[i] = nv[q];
    }
    __syncthreads();
  }
  double* yc = y + (size_t)col * ldy;
  for (int q = 0; q < PPT; ++q) {
    const int i = tid + 256 * q;
    if (i < N) yc[i] = mis[q] + gamma * u[i];
  }
}

// advection-diffusion: explicit upwind step with precomputed coefficients
template <int PPT>
__global__ __launch_bounds__(256) void k_advdiff_apply(
    int g, int steps, double inv_sig2, const double* __restrict__ coef,
    const int32_t* __restrict__ bidx, const double* __restrict__ bw, int nobs,
    const int32_t* __restrict__ slot, int nslots, const double* __restrict__ om, int ldo,
    double* __restrict__ y, int ldy, double* __restrict__ obs_store) {
  extern __shared__ double u[];
  const int N = g * g;
  const int col = blockIdx.x;
  const int tid = threadIdx.x;
  const double* v = om + (size_t)col * ldo;
  double* ob = obs_store + (size_t)col * nslots * nobs;
  const double* cC = coef;
  const double* cW = coef + N;
  const double* cE = coef + 2 * N;
  const double* cS = coef + 3 * N;
  const double* cN = coef + 4 * N;
  double nv[PPT];
  for (int q = 0; q < PPT; ++q) {
    const int i = tid + 256 * q;
    if (i < N) u[i] = v[i];
  }
  __syncthreads();
  for (int s = 1; s <= steps; ++s) {
    for (int q = 0; q < PPT; ++q) {
      const int i = tid + 256 * q;
      if (i < N) {
        const int ix = i % g, iy = i / g;
        double val = cC[i] * u[i];
        if (ix > 0) val += cW[i] * u[i - 1];
        if (ix < g - 1) val += cE[i] * u[i + 1];
        if (iy > 0) val += cS[i] * u[i - g];
        if (iy < g - 1) val += cN[i] * u[i + g];
        nv[q] = val;
      }
    }
    __syncthreads();
    for (int q = 0; q < PPT; ++q) {
      const int i = tid + 256 * q;
      if (i < N) u[i] = nv[q];
    }
    __syncthreads();
    const int sl = slot[s];
    if (sl >= 0)
      for (int o = tid; o < nobs; o += 256) {
        double acc = 0;
        for (int c = 0; c < 4; ++c) {
          const int nd = bidx[4 * o + c];
          if (nd >= 0) acc += bw[4 * o + c] * u[nd];
        }
        ob[sl * nobs + o] = acc;
      }
    __syncthreads();
  }
  for (int q = 0; q < PPT; ++q) {
    const int i = tid + 256 * q;
    if (i < N) u[i] = 0.0;
  }
  __syncthreads();
  for (int s = steps; s >= 1; --s) {
    const int sl = slot[s];
    if (sl >= 0 && tid == 0) {
      // serial scatter: several observations may share a node
      for (int o = 0; o < nobs; ++o) {
        const double d = ob[sl * nobs + o];
        for (int c = 0; c < 4; ++c) {
          const int nd = bidx[4 * o + c];
          if (nd >= 0) u[nd] += bw[4 * o + c] * d;
        }
      }
    }
    __syncthreads();
    // transpose of the step: out[j] = sum_i A[i, j] w[i]
    for (int q = 0; q < PPT; ++q) {
      const int j = tid + 256 * q;
      if (j < N) {
        const int ix = j % g, iy = j / g;
        double val = cC[j] * u[j];
        if (ix < g - 1) val += cW[j + 1] * u[j + 1];   // j is the west neighbour of j+1
        if (ix > 0) val += cE[j - 1] * u[j - 1];       // j is the east neighbour of j-1
        if (iy < g - 1) val += cS[j + g] * u[j + g];   // j is the south neighbour of j+g
        if (iy > 0) val += cN[j - g] * u[j - g];       // j is the north neighbour of j-g
        nv[q] = val;
      }
    }
    __syncthreads();
    for (int q = 0; q < PPT; ++q) {
      const int i = tid + 256 * q;
      if (i < N) u[i] = nv[q];
    }
    __syncthreads();
  }
  double* yc = y + (size_t)col * ldy;
  for (int q = 0; q < PPT; ++q) {
    const int i = tid + 256 * q;
    if (i < N) yc[i] = u[i] * inv_sig2;
  }
}

static std::vector<int32_t> slot_table(int steps, const std::vector<int>& obs) {
  std::vector<int32_t> slot(steps + 1, -1);
  for (size_t k = 0; k < obs.size(); ++k) slot[obs[k]] = (int32_t)k;
  return slot;
}

template <class F>
static void launch_ppt(int N, F&& f) {
  const int ppt = (N + 255) / 256;
  if (ppt <= 4) f(std::integral_constant<int, 4>{});
  else if (ppt <= 16) f(std::integral_constant<int, 16>{});
  else if (ppt <= 36) f(std::integral_constant<int, 36>{});
  else if (ppt <= 64) f(std::integral_constant<int, 64>{});
  else throw Error(H2_EINVAL, "grid too large for the LDS-resident sampler");
}

// ------------------------------------------------------------------ minimal surface
// Hessian of the discrete minimal-surface area (Appendix A example): heights
// on a (g+2) x (g+2) node grid, g x g interior unknowns, each cell cut along
// its anti-diagonal into a lower triangle (iy,ix),(iy,ix+1),(iy+1,ix) and an
// upper triangle (iy+1,ix+1),(iy+1,ix),(iy,ix+1); area (h^2/2) sqrt(1 + |g|^2)
// per triangle with g the leg differences / h.  Then
//   H v = sum_T B_T^T C_T B_T v,   C_T = (1/2) ((1 + |g|^2) I - g g^T) / (1 + |g|^2)^(3/2)
// with B_T the unscaled leg differences (the h factors cancel).
struct MinSurfCtx {
  int kind = 4;
  int g;
  DevBuf coef;  // per cell (cy, cx), (g+1)^2 cells: lower xx, xy, yy, upper xx, xy, yy
};

// one thread per (interior node, column): the node's rows of the six
// triangles that touch it
__global__ __launch_bounds__(256) void k_minsurf_apply(int g, int ncols,
                                                       const double* __restrict__ coef,
                                                       const double* __restrict__ om, int ldo,
                                                       double* __restrict__ y, int ldy) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  const int col = blockIdx.y;
  if (node >= g * g || col >= ncols) return;
  const int p = node / g + 1, q = node % g + 1;      // padded node coordinates
  const double* v = om + (size_t)col * ldo;
  auto V = [&](int a, int b) -> double {
    return (a >= 1 && a <= g && b >= 1 && b <= g) ? v[(size_t)(a - 1) * g + (b - 1)] : 0.0;
  };
  const int nc = g + 1;
  // lower triangle of cell (cy, cx): (qx, qy) from the legs along x and y
  auto lower = [&](int cy, int cx, double& qx, double& qy) {
    const double* c = coef + (size_t)(cy * nc + cx) * 6;
    const double o = V(cy, cx);
    const double dx = V(cy, cx + 1) - o, dy = V(cy + 1, cx) - o;
    qx = c[0] * dx + c[1] * dy;
    qy = c[1] * dx + c[2] * dy;
  };
  auto upper = [&](int cy, int cx, double& qx, double& qy) {
    const double* c = coef + (size_t)(cy * nc + cx) * 6 + 3;
    const double o = V(cy + 1, cx + 1);
    const double dx = o - V(cy + 1, cx), dy = o - V(cy, cx + 1);
    qx = c[0] * dx + c[1] * dy;
    qy = c[1] * dx + c[2] * dy;
  };
  double acc = 0.0, qx, qy;
  lower(p, q, qx, qy);         acc -= qx + qy;   // node is the right-angle corner
  lower(p, q - 1, qx, qy);     acc += qx;        // node is the corner along x
  lower(p - 1, q, qx, qy);     acc += qy;        // node is the corner along y
  upper(p - 1, q - 1, qx, qy); acc += qx + qy;   // node is the right-angle corner
  upper(p - 1, q, qx, qy);     acc -= qx;        // node is the corner back along x
  upper(p, q - 1, qx, qy);     acc -= qy;        // node is the corner back along y
  y[(size_t)col * ldy + node] = acc;
}

}  // namespace h2

using namespace h2;

extern "C" {

h2_status h2_sampler_minsurf_create(int g, const double* heights_host, void** ctx) {
  return guarded_status([&] {
    H2_CHECK(heights_host && ctx && g >= 1 && g <= 4096, H2_EINVAL,
             "bad minimal-surface sampler arguments");
    auto c = std::make_unique<MinSurfCtx>();
    c->g = g;
    const int nn = g + 2, nc = g + 1;
    const double h = 1.0 / (g + 1);
    auto M = [&](int a, int b) { return heights_host[(size_t)a * nn + b]; };
    auto set = [](double* out, double gx, double gy) {
      const double s2 = 1.0 + gx * gx + gy * gy;
      const double w = 0.5 / (s2 * std::sqrt(s2));
      out[0] = w * (1.0 + gy * gy);
      out[1] = -w * gx * gy;
      out[2] = w * (1.0 + gx * gx);
    };
    std::vector<double> coef((size_t)nc * nc * 6);
    for (int cy = 0; cy < nc; ++cy)
      for (int cx = 0; cx < nc; ++cx) {
        double* o = &coef[(size_t)(cy * nc + cx) * 6];
        set(o, (M(cy, cx + 1) - M(cy, cx)) / h, (M(cy + 1, cx) - M(cy, cx)) / h);
        set(o + 3, (M(cy + 1, cx + 1) - M(cy + 1, cx)) / h, (M(cy + 1, cx + 1) - M(cy, cx + 1)) / h);
      }
    upload(c->coef, coef);
    *ctx = c.release();
  });
}

int h2_sampler_minsurf_apply(void* ctx, int n, int ncols, const double* omega, int ld_omega,
                             double* y, int ld_y, hipStream_t stream) {
  auto* c = (MinSurfCtx*)ctx;
  if (!c || c->kind != 4 || n != c->g * c->g || ncols < 0 || ld_omega < n || ld_y < n) return 1;
  if (ncols == 0) return 0;
  if (ncols > 65535) return 1;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)ncols);
  k_minsurf_apply<<<grid, 256, 0, stream>>>(c->g, ncols, c->coef.as<double>(), omega, ld_omega, y,
                                            ld_y);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

h2_status h2_sampler_kernel_create(const double* points_host, int n, int dim, double ell,
                                   double shift, void** ctx) {
  return guarded_status([&] {
    H2_CHECK(points_host && ctx && n >= 1 && dim >= 1 && dim <= 3 && ell > 0, H2_EINVAL,
             "bad kernel sampler arguments");
    auto k = std::make_unique<KernelCtx>();
    k->n = n;
    k->dim = dim;
    k->ell = ell;
    k->shift = shift;
    std::vector<double> p((size_t)n * 3, 0.0);
    for (int i = 0; i < n; ++i)
      for (int d = 0; d < dim; ++d) p[(size_t)i * 3 + d] = points_host[(size_t)i * dim + d];
    upload(k->pts, p);
    *ctx = k.release();
  });
}

int h2_sampler_kernel_apply(void* ctx, int n, int ncols, const double* omega, int ld_omega,
                            double* y, int ld_y, hipStream_t stream) {
  auto* k = (KernelCtx*)ctx;
  if (!k || k->kind != 1 || n != k->n || ncols < 0) return 1;
  if (ncols == 0) return 0;
  dim3 grid((n + KT - 1) / KT, (ncols + KC - 1) / KC);
  k_kernel_apply<<<grid, 256, 0, stream>>>(n, ncols, k->pts.as<double>(), 1.0 / k->ell, k->shift,
                                           omega, ld_omega, y, ld_y);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

h2_status h2_sampler_kernel_batched_create(int nprob, const int64_t* row_off_host,
                                           const double* points_host, int dim,
                                           const double* ell_host, const double* shift_host,
                                           void** ctx) {
  return guarded_status([&] {
    H2_CHECK(nprob >= 1 && row_off_host && points_host && ell_host && shift_host && ctx &&
             dim >= 1 && dim <= 3, H2_EINVAL, "bad batched kernel sampler arguments");
    H2_CHECK(row_off_host[0] == 0, H2_EINVAL, "row offsets must start at 0");
    auto k = std::make_unique<KernelBatchCtx>();
    k->nprob = nprob;
    k->off.assign(row_off_host, row_off_host + nprob + 1);
    const int64_t rows = k->off[nprob];
    std::vector<double> p((size_t)rows * 3, 0.0), prm(2 * (size_t)nprob);
    std::vector<int32_t> tiles;
    for (int i = 0; i < nprob; ++i) {
      H2_CHECK(k->off[i + 1] > k->off[i] && ell_host[i] > 0, H2_EINVAL,
               "empty problem or non-positive length scale");
      prm[2 * i] = 1.0 / ell_host[i];
      prm[2 * i + 1] = shift_host[i];
      for (int64_t r0 = 0; r0 < k->off[i + 1] - k->off[i]; r0 += KT) {
        tiles.push_back(i);
        tiles.push_back((int32_t)r0);
      }
    }
    for (int64_t r = 0; r < rows; ++r)
      for (int d = 0; d < dim; ++d) p[(size_t)r * 3 + d] = points_host[(size_t)r * dim + d];
    k->ntiles = (int)(tiles.size() / 2);
    upload(k->pts, p);
    upload(k->tiles, tiles);
    upload(k->prm, prm);
    std::vector<int64_t> off(k->off);
    DevBuf doff;
    upload(doff, off);
    k->tiles_off = std::move(doff);
    *ctx = k.release();
  });
}

int h2_sampler_kernel_batched_apply(void* ctx, int nprob, const int64_t* row_off,
                                    const int32_t* active, int ncols, const double* omega, int ld,
                                    double* y, hipStream_t stream) {
  auto* k = (KernelBatchCtx*)ctx;
  if (!k || k->kind != 5 || nprob != k->nprob || !row_off || ncols < 0) return 1;
  for (int i = 0; i <= nprob; ++i)
    if (row_off[i] != k->off[i]) return 1;
  if (ld < k->off[nprob]) return 1;
  (void)active;  // inactive problems have zero rows in omega: their products are zero
  if (ncols == 0) return 0;
  dim3 grid((unsigned)k->ntiles, (unsigned)((ncols + KC - 1) / KC));
  k_kernel_apply_batched<<<grid, 256, 0, stream>>>(k->tiles.as<int32_t>(),
                                                   k->tiles_off.as<int64_t>(), k->prm.as<double>(),
                                                   k->pts.as<double>(), ncols, omega, ld, y);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

h2_status h2_sampler_diffusion_create(int g, double kappa, double dt, int steps,
                                      const int32_t* obs_steps, int n_obs_steps,
                                      const int32_t* obs_index, int obs_count, double sigma,
                                      double gamma, double beta, void** ctx) {
  return guarded_status([&] {
    H2_CHECK(ctx && g >= 2 && g <= 128 && steps >= 1 && sigma > 0, H2_EINVAL,
             "bad diffusion sampler arguments");
    H2_CHECK(n_obs_steps >= 1 && obs_steps && obs_count >= 1 && obs_index, H2_EINVAL,
             "observations required");
    auto c = std::make_unique<StepCtx>();
    c->kind = 2;
    c->g = g;
    c->steps = steps;
    const double h = 1.0 / (g + 1);
    c->cdiff = dt * kappa / (h * h);
    c->sigma = sigma;
    c->gamma = gamma;
    c->beta_h2 = beta / (h * h);
    for (int i = 0; i < n_obs_steps; ++i) {
      H2_CHECK(obs_steps[i] >= 1 && obs_steps[i] <= steps, H2_EINVAL, "observation step range");
      c->obs_steps.push_back(obs_steps[i]);
    }
    std::vector<int32_t> idx;
    for (int a = 0; a < obs_count; ++a)
      for (int b = 0; b < obs_count; ++b) {
        H2_CHECK(obs_index[a] >= 0 && obs_index[a] < g && obs_index[b] >= 0 && obs_index[b] < g,
                 H2_EINVAL, "observation index range");
        idx.push_back(obs_index[a] * g + obs_index[b]);   // (row iy, column ix)
      }
    c->nobs = (int)idx.size();
    upload(c->obs_idx, idx);
    upload(c->obs_step_flag, slot_table(steps, c->obs_steps));
    *ctx = c.release();
  });
}

int h2_sampler_diffusion_apply(void* ctx, int n, int ncols, const double* omega, int ld_omega,
                               double* y, int ld_y, hipStream_t stream) {
  auto* c = (StepCtx*)ctx;
  if (!c || c->kind != 2 || n != c->g * c->g || ncols < 0) return 1;
  if (ncols == 0) return 0;
  try {
    const int nslots = (int)c->obs_steps.size();
    c->work.reserve((size_t)ncols * nslots * c->nobs * sizeof(double));
    const size_t lds = (size_t)n * sizeof(double);
    launch_ppt(n, [&](auto P) {
      auto kfn = k_diffusion_apply<decltype(P)::value>;
      if (lds > 65536)
        H2_HIP(hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      kfn<<<ncols, 256, lds, stream>>>(
          c->g, c->steps, c->cdiff, 1.0 / (c->sigma * c->sigma), c->gamma, c->beta_h2,
          c->obs_idx.as<int32_t>(), c->nobs, c->obs_step_flag.as<int32_t>(), nslots, omega,
          ld_omega, y, ld_y, c->work.as<double>());
    });
  } catch (...) {
    return 3;
  }
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

h2_status h2_sampler_advdiff_create(int g, double kappa, int steps, const int32_t* obs_steps,
                                    int n_obs_steps, const double* obs_points_host, int n_obs,
                                    double sigma, const int32_t* mode_a, const int32_t* mode_b,
                                    const double* mode_s, int n_modes, void** ctx) {
  return guarded_status([&] {
    H2_CHECK(ctx && g >= 2 && g <= 128 && steps >= 1 && sigma > 0 && kappa > 0, H2_EINVAL,
             "bad advdiff sampler arguments");
    H2_CHECK(obs_steps && n_obs_steps >= 1 && obs_points_host && n_obs >= 1, H2_EINVAL,
             "observations required");
    auto c = std::make_unique<StepCtx>();
    c->kind = 3;
    c->g = g;
    c->steps = steps;
    c->sigma = sigma;
    const double h = 1.0 / (g + 1), PI = 3.141592653589793;
    const int N = g * g;
    // velocity v = (d psi / dy, -d psi / dx), psi = sum s sin(pi a x) sin(pi b y)
    std::vector<double> vx(N, 0.0), vy(N, 0.0);
    for (int iy = 0; iy < g; ++iy)
      for (int ix = 0; ix < g; ++ix) {
        const double x = (ix + 1) * h, yy = (iy + 1) * h;
        double ax = 0, ay = 0;
        for (int m = 0; m < n_modes; ++m) {
          const double a = mode_a[m], b = mode_b[m], s = mode_s[m];
          ax += s * std::sin(PI * a * x) * PI * b * std::cos(PI * b * yy);
          ay -= s * PI * a * std::cos(PI * a * x) * std::sin(PI * b * yy);
        }
        vx[iy * g + ix] = ax;
        vy[iy * g + ix] = ay;
      }
    double vmax = 0;
    for (int i = 0; i < N; ++i) vmax = std::max(vmax, std::fabs(vx[i]) + std::fabs(vy[i]));
    const double dt = 0.5 * std::min(vmax > 0 ? h / vmax : 1e300, h * h / (4.0 * kappa));
    const double d = kappa / (h * h);
    std::vector<double> coef((size_t)5 * N);
    for (int i = 0; i < N; ++i) {
      const double cxm = vx[i] > 0 ? vx[i] / h : 0.0, cxp = vx[i] > 0 ? 0.0 : -vx[i] / h;
      const double cym = vy[i] > 0 ? vy[i] / h : 0.0, cyp = vy[i] > 0 ? 0.0 : -vy[i] / h;
      coef[i] = 1.0 + dt * (-4.0 * d - cxm - cxp - cym - cyp);
      coef[N + i] = dt * (d + cxm);
      coef[2 * N + i] = dt * (d + cxp);
      coef[3 * N + i] = dt * (d + cym);
      coef[4 * N + i] = dt * (d + cyp);
    }
    upload(c->coef, coef);
    std::vector<int32_t> bidx((size_t)4 * n_obs, -1);
    std::vector<double> bw((size_t)4 * n_obs, 0.0);
    for (int o = 0; o < n_obs; ++o) {
      const double fx = obs_points_host[2 * o] / h, fy = obs_points_host[2 * o + 1] / h;
      const int i0 = (int)std::floor(fx), j0 = (int)std::floor(fy);
      const double tx = fx - i0, ty = fy - j0;
      int q = 0;
      for (int di = 0; di < 2; ++di)
        for (int dj = 0; dj < 2; ++dj) {
          const double wx = di ? tx : 1 - tx, wy = dj ? ty : 1 - ty;
          const int ii = i0 + di, jj = j0 + dj;
          if (ii >= 1 && ii <= g && jj >= 1 && jj <= g && wx * wy != 0.0) {
            bidx[4 * o + q] = (jj - 1) * g + (ii - 1);
            bw[4 * o + q] = wx * wy;
          }
          ++q;
        }
    }
    c->nobs = n_obs;
    upload(c->bil_idx, bidx);
    upload(c->bil_w, bw);
    for (int i = 0; i < n_obs_steps; ++i) {
      H2_CHECK(obs_steps[i] >= 1 && obs_steps[i] <= steps, H2_EINVAL, "observation step range");
      c->obs_steps.push_back(obs_steps[i]);
    }
    upload(c->obs_step_flag, slot_table(steps, c->obs_steps));
    *ctx = c.release();
  });
}

int h2_sampler_advdiff_apply(void* ctx, int n, int ncols, const double* omega, int ld_omega,
                             double* y, int ld_y, hipStream_t stream) {
  auto* c = (StepCtx*)ctx;
  if (!c || c->kind != 3 || n != c->g * c->g || ncols < 0) return 1;
  if (ncols == 0) return 0;
  try {
    const int nslots = (int)c->obs_steps.size();
    c->work.reserve((size_t)ncols * nslots * c->nobs * sizeof(double));
    const size_t lds = (size_t)n * sizeof(double);
    launch_ppt(n, [&](auto P) {
      auto kfn = k_advdiff_apply<decltype(P)::value>;
      if (lds > 65536)
        H2_HIP(hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      kfn<<<ncols, 256, lds, stream>>>(
          c->g, c->steps, 1.0 / (c->sigma * c->sigma), c->coef.as<double>(),
          c->bil_idx.as<int32_t>(), c->bil_w.as<double>(), c->nobs, c->obs_step_flag.as<int32_t>(),
          nslots, omega, ld_omega, y, ld_y, c->work.as<double>());
    });
  } catch (...) {
    return 3;
  }
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

void h2_sampler_destroy(void* ctx) {
  if (!ctx) return;
  const int kind = *(int*)ctx;
  if (kind == 1) delete (KernelCtx*)ctx;
  else if (kind == 4) delete (MinSurfCtx*)ctx;
  else if (kind == 5) delete (KernelBatchCtx*)ctx;
  else delete (StepCtx*)ctx;
}

}  // extern "C"
