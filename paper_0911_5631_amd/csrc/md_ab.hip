// md_ab.hip -- the Newton's-third-law A/B of the force phase.
//
// The paper drops Newton's third law on the GPU (Sec. 3.3): every atom keeps
// the full list of its neighbours and sums only its own force, so no two
// threads ever write one location.  The CPU form it gives up keeps each pair
// once and adds the reaction to the partner (Sec. 3.2).  These kernels put
// both forms side by side on gfx950 with one plain structure: a list over the
// cell-sorted storage (entries are storage indices with the image code, no
// LDS window), built full (every j != i) or half (j > i in storage order,
// each pair once), and a force loop that either keeps its sum in registers
// (full) or also adds -f d to the partner with FP32 atomics (half).  The
// production step kernel is the tuned form of the full side.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "md_device.h"
#include "md_kernels.h"

namespace md {

namespace {

// Cell coordinate of one of the 27 offsets wrapped into [0, G), and the
// image code of the atoms found there (reading 6: -L past G-1, +L below 0).
__device__ __forceinline__ int ab_wrap(int c, int G, uint32_t *code) {
  if (c >= G) {
    *code = 3;
    return c - G;
  }
  if (c < 0) {
    *code = 1;
    return c + G;
  }
  *code = 0;
  return c;
}

__device__ __forceinline__ double ab_shift(uint32_t code, double L) {
  return code == 0 ? 0.0 : (code == 1 ? L : -L);
}

// One thread per atom i (storage order): the 27 cells around i's cell,
// offsets z-major and x fastest, each cell's atoms in storage order; keep j
// with r^2 < r_n^2 (FP64, no FMA) and, for the half list, j > i.
template <bool HALF>
__global__ __launch_bounds__(TILE) void k_ab_build(const double *__restrict__ x,
                                                  const double *__restrict__ y,
                                                  const double *__restrict__ z,
                                                  const int32_t *__restrict__ cell,
                                                  const int32_t *__restrict__ cs, int n, int npad,
                                                  int G, double L, double rn2, int mcap,
                                                  int32_t *__restrict__ W, int32_t *__restrict__ m,
                                                  int32_t *__restrict__ overflow) {
  const int i = blockIdx.x * TILE + threadIdx.x;
  if (i >= n) return;
  const double xi = x[i], yi = y[i], zi = z[i];
  const int c = cell[i];
  const int cx = c % G, cy = (c / G) % G, cz = c / (G * G);
  int cnt = 0;
  for (int oz = -1; oz <= 1; ++oz) {
    uint32_t kz;
    const int nz = ab_wrap(cz + oz, G, &kz);
    const double bz = ab_shift(kz, L);
    for (int oy = -1; oy <= 1; ++oy) {
      uint32_t ky;
      const int ny = ab_wrap(cy + oy, G, &ky);
      const double by = ab_shift(ky, L);
      for (int ox = -1; ox <= 1; ++ox) {
        uint32_t kx;
        const int nx = ab_wrap(cx + ox, G, &kx);
        const double bx = ab_shift(kx, L);
        const uint32_t code = kx | (ky << 2) | (kz << 4);
        const int cc = (nz * G + ny) * G + nx;
        const int lo = cs[cc], hi = cs[cc + 1];
        for (int j = HALF ? max(lo, i + 1) : lo; j < hi; ++j) {
          if (!HALF && j == i) continue;
          const double dx = (xi - x[j]) + bx, dy = (yi - y[j]) + by, dz = (zi - z[j]) + bz;
          const double s = (dx * dx + dy * dy) + dz * dz;
          if (s < rn2) {
            if (cnt < mcap) W[(size_t)cnt * npad + i] = (int32_t)((uint32_t)j | (code << J_BITS));
            ++cnt;
          }
        }
      }
    }
  }
  m[i] = min(cnt, mcap);
  if (cnt > mcap) atomicAdd(overflow, 1);
}

// The cell-centric build of the earlier GPU codes (the organisation the
// paper describes at the end of Sec. 3.4 and times as "old" in Table 3):
// one workgroup per cell, one thread per occupant (layer l of H_{c,l}) of
// the cell.  For each of the 27 neighbouring cells in turn the workgroup
// loads that cell's atoms into LDS and every thread tests its own atom
// against them.  Only the cell's occupants have work (a few for the soft
// spheres, up to ~50 for the longest LJ cutoff), so most lanes of the wave
// idle: the scaling limit the paper points out.  Entries come in the order
// of k_ab_build<false> (offsets z-major, x fastest; ascending storage index
// within a cell), so the two lists are identical.
__global__ __launch_bounds__(64) void k_ab_build_cells(const double *__restrict__ x,
                                                      const double *__restrict__ y,
                                                      const double *__restrict__ z,
                                                      const int32_t *__restrict__ cs, int npad,
                                                      int G, double L, double rn2, int mcap,
                                                      int32_t *__restrict__ W,
                                                      int32_t *__restrict__ m,
                                                      int32_t *__restrict__ overflow) {
  __shared__ double sx[64], sy[64], sz[64];
  const int c = blockIdx.x;
  const int lo = cs[c], cnt = cs[c + 1] - lo;
  const int cx = c % G, cy = (c / G) % G, cz = c / (G * G);
  for (int l0 = 0; l0 < cnt; l0 += 64) {  // cells of more than 64 occupants in chunks
    const bool own = l0 + (int)threadIdx.x < cnt;
    const int i = lo + l0 + threadIdx.x;
    double xi = 0.0, yi = 0.0, zi = 0.0;
    if (own) {
      xi = x[i];
      yi = y[i];
      zi = z[i];
    }
    int k = 0;
    for (int oz = -1; oz <= 1; ++oz) {
      uint32_t kz;
      const int nz = ab_wrap(cz + oz, G, &kz);
      const double bz = ab_shift(kz, L);
      for (int oy = -1; oy <= 1; ++oy) {
        uint32_t ky;
        const int ny = ab_wrap(cy + oy, G, &ky);
        const double by = ab_shift(ky, L);
        for (int ox = -1; ox <= 1; ++ox) {
          uint32_t kx;
          const int nx = ab_wrap(cx + ox, G, &kx);
          const double bx = ab_shift(kx, L);
          const uint32_t code = kx | (ky << 2) | (kz << 4);
          const int cc = (nz * G + ny) * G + nx;
          const int lo2 = cs[cc], cnt2 = cs[cc + 1] - lo2;
          for (int j0 = 0; j0 < cnt2; j0 += 64) {
            __syncthreads();
            if (j0 + (int)threadIdx.x < cnt2) {
              sx[threadIdx.x] = x[lo2 + j0 + threadIdx.x];
              sy[threadIdx.x] = y[lo2 + j0 + threadIdx.x];
              sz[threadIdx.x] = z[lo2 + j0 + threadIdx.x];
            }
            __syncthreads();
            const int nj = min(64, cnt2 - j0);
            if (own) {
              for (int q = 0; q < nj; ++q) {
                const int j = lo2 + j0 + q;
                if (j == i) continue;
                const double dx = (xi - sx[q]) + bx, dy = (yi - sy[q]) + by,
                             dz = (zi - sz[q]) + bz;
                const double s = (dx * dx + dy * dy) + dz * dz;
                if (s < rn2) {
                  if (k < mcap) W[(size_t)k * npad + i] = (int32_t)((uint32_t)j | (code << J_BITS));
                  ++k;
                }
              }
            }
          }
        }
      }
    }
    if (own) {
      m[i] = min(k, mcap);
      if (k > mcap) atomicAdd(overflow, 1);
    }
  }
}

// One thread per atom i: Eq. (1) (with the soft-sphere shift only in the
// energy, not computed here) in FP32 on FP64 separations, for the entries of
// i's list.  Full: the sum is i's force, stored once.  Half: the reaction
// -f d goes to the partner by atomics, and i's own sum is added last (F must
// be zero before the launch).
template <bool HALF>
__global__ __launch_bounds__(TILE) void k_ab_forces(const double *__restrict__ x,
                                                   const double *__restrict__ y,
                                                   const double *__restrict__ z,
                                                   const int32_t *__restrict__ W,
                                                   const int32_t *__restrict__ m, int n, int npad,
                                                   double L, double rc2, float *__restrict__ F) {
  const int i = blockIdx.x * TILE + threadIdx.x;
  if (i >= n) return;
  const double xi = x[i], yi = y[i], zi = z[i];
  float fx = 0.f, fy = 0.f, fz = 0.f;
  const int mi = m[i];
  for (int q = 0; q < mi; ++q) {
    const uint32_t e = (uint32_t)W[(size_t)q * npad + i];
    const int j = (int)(e & IDX_MASK);
    const double dx = (xi - x[j]) + (double)((int32_t)(e << (32 - J_BITS - 2)) >> 30) * L;
    const double dy = (yi - y[j]) + (double)((int32_t)(e << (32 - J_BITS - 4)) >> 30) * L;
    const double dz = (zi - z[j]) + (double)((int32_t)e >> 30) * L;
    const double s = (dx * dx + dy * dy) + dz * dz;
    if (s < rc2) {
      const float sr = (float)s;
      const float r0 = __builtin_amdgcn_rcpf(sr);  // refined as the step kernel does
      const float rri = __builtin_fmaf(r0, __builtin_fmaf(-sr, r0, 1.0f), r0);
      const float rri3 = rri * rri * rri;
      const float f = 48.f * rri3 * (rri3 - 0.5f) * rri;
      const float ax = f * (float)dx, ay = f * (float)dy, az = f * (float)dz;
      fx += ax;
      fy += ay;
      fz += az;
      if (HALF) {
        unsafeAtomicAdd(&F[j], -ax);
        unsafeAtomicAdd(&F[npad + j], -ay);
        unsafeAtomicAdd(&F[2 * (size_t)npad + j], -az);
      }
    }
  }
  if (HALF) {
    unsafeAtomicAdd(&F[i], fx);
    unsafeAtomicAdd(&F[npad + i], fy);
    unsafeAtomicAdd(&F[2 * (size_t)npad + i], fz);
  } else {
    F[i] = fx;
    F[npad + i] = fy;
    F[2 * (size_t)npad + i] = fz;
  }
}

// Zero `words` 32-bit words (a fill kernel rather than a memset node).
__global__ __launch_bounds__(TILE) void k_ab_zero(uint32_t *__restrict__ p, size_t words) {
  for (size_t q = (size_t)blockIdx.x * TILE + threadIdx.x; q < words;
       q += (size_t)gridDim.x * TILE)
    p[q] = 0u;
}

// The forces in the caller's order (out[3 id + a], FP64) and the total list
// length (added to *entries, which must be zero before the launch).
__global__ __launch_bounds__(TILE) void k_ab_output(const float *__restrict__ F,
                                                   const int32_t *__restrict__ id,
                                                   const int32_t *__restrict__ m, int n, int npad,
                                                   double *__restrict__ out,
                                                   unsigned long long *entries) {
  const int p = blockIdx.x * TILE + threadIdx.x;
  unsigned long long k = 0;
  if (p < n) {
    const int i = id[p];
    if (i >= 0 && i < n)
      for (int a = 0; a < 3; ++a) out[3 * (size_t)i + a] = (double)F[(size_t)a * npad + p];
    k = (unsigned long long)m[p];
  }
  for (int o = 32; o > 0; o >>= 1) k += __shfl_xor(k, o, 64);
  if ((threadIdx.x & 63) == 0 && k) atomicAdd(entries, k);
}

}  // namespace

void launch_ab_zero(void *p, size_t bytes, hipStream_t s) {
  const size_t words = bytes / 4;
  const size_t blocks = std::min<size_t>((words + TILE - 1) / TILE, 4096);
  hipLaunchKernelGGL(k_ab_zero, dim3((unsigned)std::max<size_t>(blocks, 1)), dim3(TILE), 0, s,
                     (uint32_t *)p, words);
}

void launch_ab_output(const float *F, const int32_t *id, const int32_t *m, int n, int npad,
                      double *out, unsigned long long *entries, hipStream_t s) {
  hipLaunchKernelGGL(k_ab_output, dim3((n + TILE - 1) / TILE), dim3(TILE), 0, s, F, id, m, n,
                     npad, out, entries);
}

void launch_ab_build(bool half, const double *x, const double *y, const double *z,
                     const int32_t *cell, const int32_t *cs, int n, int npad, int G, double L,
                     double rn2, int mcap, int32_t *W, int32_t *m, int32_t *overflow,
                     hipStream_t s) {
  const dim3 grid((n + TILE - 1) / TILE);
  if (half)
    hipLaunchKernelGGL(k_ab_build<true>, grid, dim3(TILE), 0, s, x, y, z, cell, cs, n, npad, G,
                       L, rn2, mcap, W, m, overflow);
  else
    hipLaunchKernelGGL(k_ab_build<false>, grid, dim3(TILE), 0, s, x, y, z, cell, cs, n, npad, G,
                       L, rn2, mcap, W, m, overflow);
}

void launch_ab_build_cells(const double *x, const double *y, const double *z, const int32_t *cs,
                           int npad, int G, double L, double rn2, int mcap, int32_t *W,
                           int32_t *m, int32_t *overflow, hipStream_t s) {
  hipLaunchKernelGGL(k_ab_build_cells, dim3(G * G * G), dim3(64), 0, s, x, y, z, cs, npad, G, L,
                     rn2, mcap, W, m, overflow);
}

void launch_ab_forces(bool half, const double *x, const double *y, const double *z,
                      const int32_t *W, const int32_t *m, int n, int npad, double L, double rc2,
                      float *F, hipStream_t s) {
  const dim3 grid((n + TILE - 1) / TILE);
  if (half)
    hipLaunchKernelGGL(k_ab_forces<true>, grid, dim3(TILE), 0, s, x, y, z, W, m, n, npad, L, rc2,
                       F);
  else
    hipLaunchKernelGGL(k_ab_forces<false>, grid, dim3(TILE), 0, s, x, y, z, W, m, n, npad, L,
                       rc2, F);
}

}  // namespace md
