// GPW route of the diffuse (DD) pair densities: appendix "Evaluation of density
// on real space grid (GPW)" and section "Density classification: compact and
// diffuse" (the DD densities are Fourier transformed through a real-space grid).
//
//   rho_D(r)  = sum_{DD pairs, images T} w D_ab(L) c_a c_b N_a N_b K
//               e^{-p |X|^2} (X + P - A)^a (X + P - B)^b,     X = r - P - T
//               on the uniform grid r = sum_i (j_i / N_i) a_i of the cell,
//   rho_D(G)  = (1/N) sum_r rho_D(r) e^{-i G.r}                 for G in the set,
//   V_D(r)    = sum_{G in the set} V_D(G) e^{i G.r},
//   J_ab(L)  += c_a c_b N_a N_b K (Omega/N) sum_{r, T} V_D(r) e^{-p |X|^2} (...)^a (...)^b.
//
// Both sums over the grid are the transforms of the analytic route up to
// aliasing: with G = B n and r on the grid, G.r = 2 pi sum_i n_i j_i / N_i, so the
// transform is separable along the lattice axes for any cell (three passes of
// one-dimensional sums restricted to the |n_i| <= M_i the G set needs), and with
// N_i = 2 ceil(1.25 M_i) + 1 every G of the set aliases only onto vectors outside
// the cutoff sphere, where a DD density (p < omega^2) has decayed below the
// long-range kernel's cutoff weight.
//
// The pair product is written as one Gaussian at P (eq. "Gaussian product of the
// radial decay") with the Cartesian factors taken about its two centres; every
// sum runs in a fixed order (no atomics): the collocation gathers per grid point
// over the image entries of its tile, the integration reduces per DD pair.
#include <hip/hip_runtime.h>

#include "kernel_common.h"
#include "kernels.h"

namespace pwdf {

constexpr double kPiG = 3.14159265358979323846;

// Cartesian component idx of an l shell, descending lexicographic (lx, ly, lz)
__device__ __forceinline__ void gpw_cart(int l, int idx, int &x, int &y, int &z) {
  int n = 0;
  for (int a = l; a >= 0; --a)
    for (int b = l - a; b >= 0; --b) {
      if (n == idx) {
        x = a;
        y = b;
        z = l - a - b;
        return;
      }
      ++n;
    }
  x = y = z = 0;
}

// position of grid point j and of the lattice translation m
__device__ __forceinline__ void gpw_point(const Dev &d, int j0, int j1, int j2, double (&r)[3]) {
  const double f0 = (double)j0 / d.gN[0], f1 = (double)j1 / d.gN[1], f2 = (double)j2 / d.gN[2];
#pragma unroll
  for (int c = 0; c < 3; ++c) r[c] = d.lat[c * 3 + 0] * f0 + d.lat[c * 3 + 1] * f1 + d.lat[c * 3 + 2] * f2;
}

// c_a c_b N_a N_b K of a pair: the analytic prefactor pref_j = 2 c c N N K (pi/p)^{3/2}
// without its transform factor and its half-space 2
__device__ __forceinline__ double gpw_pref(const PairAux &x) {
  const double s = kPiG / x.p;
  return 0.5 * x.pref_j / (s * sqrt(s));
}

// One image entry of a DD pair as the collocation reads it: the Gaussian's centre
// P + T, its squared cut radius and exponent, the pair's weight w c c N N K, the
// offsets P - A and P - B, the grid box, the shells' l and the D(L) block offset.
struct GpwEnt {
  double cx, cy, cz, rc2, p, coef;
  double xpa[3], xpb[3];
  int box[6];
  int la, lb;
  int64_t eoff;
};

constexpr int kGpwBatch = 64;  // image entries staged in LDS at a time

// rho_D on the grid, one workgroup per work item (a run of one tile's image
// entries; 8^3 points, two per thread): the entries are staged in LDS in batches
// (one thread per entry gathers its pair data), then every thread adds the
// batch's entries to its points in list order.  The item's partial tile goes to
// grid_p; k_gpw_collect sums a tile's items in order.
__global__ __launch_bounds__(256) void k_gpw_collocate(const Dev d) {
  __shared__ GpwEnt se[kGpwBatch];
  const int item = blockIdx.x, dm = blockIdx.y;
  const int t = d.gitem[3 * item], e0 = d.gitem[3 * item + 1], e1 = d.gitem[3 * item + 2];
  const int t0 = t % d.gtiles[0], t1 = (t / d.gtiles[0]) % d.gtiles[1], t2 = t / (d.gtiles[0] * d.gtiles[1]);
  const double *Dblk = d.Dblk + (size_t)dm * d.nelem;
  int jj[2][3];
  double r[2][3], rho[2] = {0.0, 0.0};
  bool in[2];
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    const int u = threadIdx.x + 256 * v;
    jj[v][0] = t0 * 8 + (u & 7);
    jj[v][1] = t1 * 8 + ((u >> 3) & 7);
    jj[v][2] = t2 * 8 + (u >> 6);
    in[v] = jj[v][0] < d.gN[0] && jj[v][1] < d.gN[1] && jj[v][2] < d.gN[2];
    gpw_point(d, jj[v][0], jj[v][1], jj[v][2], r[v]);
  }
  for (int b0 = e0; b0 < e1; b0 += kGpwBatch) {
    const int nb = min(kGpwBatch, e1 - b0);
    __syncthreads();
    if ((int)threadIdx.x < nb) {
      const int ent = d.gtile_ent[b0 + threadIdx.x];
      const int k = d.gimg[4 * ent], m0 = d.gimg[4 * ent + 1], m1 = d.gimg[4 * ent + 2], m2 = d.gimg[4 * ent + 3];
      const int q = d.dd_q[k];
      const BlockRec b = d.blocks[d.dd_blk[k]];
      const PairAux x = d.aux[q];
      GpwEnt g;
      g.cx = d.gP[4 * k + 0] + d.lat[0] * m0 + d.lat[1] * m1 + d.lat[2] * m2;
      g.cy = d.gP[4 * k + 1] + d.lat[3] * m0 + d.lat[4] * m1 + d.lat[5] * m2;
      g.cz = d.gP[4 * k + 2] + d.lat[6] * m0 + d.lat[7] * m1 + d.lat[8] * m2;
      g.rc2 = d.gP[4 * k + 3];
      g.p = x.p;
      g.coef = x.w * gpw_pref(x);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        g.xpa[c] = x.xpa[c];
        g.xpb[c] = x.xpb[c];
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) g.box[c] = d.gimg_box[6 * (size_t)ent + c];
      g.la = d.sh_l[b.sa];
      g.lb = d.sh_l[b.sb];
      g.eoff = b.eoff;
      se[threadIdx.x] = g;
    }
    __syncthreads();
    for (int e = 0; e < nb; ++e) {
      const GpwEnt &g = se[e];
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        if (!in[v] || jj[v][0] < g.box[0] || jj[v][0] > g.box[1] || jj[v][1] < g.box[2] || jj[v][1] > g.box[3] ||
            jj[v][2] < g.box[4] || jj[v][2] > g.box[5])
          continue;
        const double X[3] = {r[v][0] - g.cx, r[v][1] - g.cy, r[v][2] - g.cz};
        const double x2 = X[0] * X[0] + X[1] * X[1] + X[2] * X[2];
        if (x2 > g.rc2) continue;
        double pa[3][kMaxL + 1], pb[3][kMaxL + 1];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          pa[c][0] = pb[c][0] = 1.0;
#pragma unroll
          for (int l = 1; l <= kMaxL; ++l) {
            pa[c][l] = pa[c][l - 1] * (X[c] + g.xpa[c]);
            pb[c][l] = pb[c][l - 1] * (X[c] + g.xpb[c]);
          }
        }
        const int ncb = ncart(g.lb);
        double sum = 0.0;
        for (int ia = 0; ia < ncart(g.la); ++ia) {
          int ax, ay, az;
          gpw_cart(g.la, ia, ax, ay, az);
          const double fa = pa[0][ax] * pa[1][ay] * pa[2][az];
          for (int ib = 0; ib < ncb; ++ib) {
            int bx, by, bz;
            gpw_cart(g.lb, ib, bx, by, bz);
            sum = fma(Dblk[g.eoff + ia * ncb + ib] * fa, pb[0][bx] * pb[1][by] * pb[2][bz], sum);
          }
        }
        rho[v] = fma(g.coef * exp(-g.p * x2), sum, rho[v]);
      }
    }
  }
  double *out = d.grid_p + ((size_t)dm * d.ngitems + item) * 512;
  out[threadIdx.x] = rho[0];
  out[threadIdx.x + 256] = rho[1];
}

// rho_D of a tile: its work items' partial tiles summed in item order
__global__ __launch_bounds__(256) void k_gpw_collect(const Dev d) {
  const int t = blockIdx.x, dm = blockIdx.y;
  const int t0 = t % d.gtiles[0], t1 = (t / d.gtiles[0]) % d.gtiles[1], t2 = t / (d.gtiles[0] * d.gtiles[1]);
  const int i0 = d.gitem_off[t], i1 = d.gitem_off[t + 1];
  for (int u = threadIdx.x; u < 512; u += 256) {
    const int j0 = t0 * 8 + (u & 7), j1 = t1 * 8 + ((u >> 3) & 7), j2 = t2 * 8 + (u >> 6);
    if (j0 >= d.gN[0] || j1 >= d.gN[1] || j2 >= d.gN[2]) continue;
    double s = 0.0;
    for (int i = i0; i < i1; ++i) s += d.grid_p[((size_t)dm * d.ngitems + i) * 512 + u];
    d.grid_r[(size_t)dm * d.gpts + ((size_t)j2 * d.gN[1] + j1) * d.gN[0] + j0] = s;
  }
}

// One pass of the separable transform along axis a: out[o2][o1][o0] (dims d0, d1,
// d2) = sum_t in[..t on axis a..] e^{sign 2 pi i n j / N}, where forward passes
// (out index k on axis a) take n = k - M, j = t, and inverse passes (out index j)
// take n = t - M, j = o_a.  The input has the output's dims except nin along a;
// rin / rout: real input (first forward pass) / real output (last inverse pass,
// the real part).  Thread per output element, t in order.
__global__ __launch_bounds__(256) void k_gpw_axis(const double2 *__restrict__ in, const double *__restrict__ rin,
                                                  double2 *__restrict__ out, double *__restrict__ rout, int d0,
                                                  int d1, int d2, int a, int nin, int N, int M, int sign,
                                                  int forward) {
  const int64_t nout = (int64_t)d0 * d1 * d2;
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int dm = blockIdx.y;
  if (o >= nout) return;
  int oi[3];
  oi[0] = (int)(o % d0);
  oi[1] = (int)((o / d0) % d1);
  oi[2] = (int)(o / ((int64_t)d0 * d1));
  int di[3] = {d0, d1, d2};
  di[a] = nin;
  const int64_t nin_tot = (int64_t)di[0] * di[1] * di[2];
  int64_t stride = 1;
  for (int i = 0; i < a; ++i) stride *= di[i];
  int ii[3] = {oi[0], oi[1], oi[2]};
  ii[a] = 0;
  const int64_t base = ((int64_t)ii[2] * di[1] + ii[1]) * di[0] + ii[0] + (int64_t)dm * nin_tot;
  double sr = 0.0, si = 0.0;
  for (int t = 0; t < nin; ++t) {
    const int n = forward ? oi[a] - M : t - M, j = forward ? t : oi[a];
    int r = (int)(((int64_t)n * j) % N);
    if (r < 0) r += N;
    double sn, cs;
    sincospi(2.0 * r / N, &sn, &cs);
    sn *= sign;
    double xr, xi;
    if (rin) {
      xr = rin[base + t * stride];
      xi = 0.0;
    } else {
      const double2 v = in[base + t * stride];
      xr = v.x;
      xi = v.y;
    }
    sr = fma(xr, cs, fma(-xi, sn, sr));
    si = fma(xr, sn, fma(xi, cs, si));
  }
  if (rout)
    rout[(int64_t)dm * nout + o] = sr;
  else
    out[(int64_t)dm * nout + o] = make_double2(sr, si);
}

// rho_D per slot from the transformed grid (1/N of the sum); padding slots 0
__global__ __launch_bounds__(256) void k_gpw_to_slots(const Dev d) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x, dm = blockIdx.y;
  if (slot >= d.nslot) return;
  double2 v = make_double2(0.0, 0.0);
  if (d.slot_v[slot] != 0.0) {
    const int K0 = 2 * d.gM[0] + 1, K1 = 2 * d.gM[1] + 1, K2 = 2 * d.gM[2] + 1;
    const int *n = d.slot_miller + 3 * (size_t)slot;
    const double2 c = d.grid_c[(size_t)dm * K0 * K1 * K2 +
                               ((size_t)(n[2] + d.gM[2]) * K1 + (n[1] + d.gM[1])) * K0 + (n[0] + d.gM[0])];
    v = make_double2(c.x / d.gpts, c.y / d.gpts);
  }
  d.rhoD[(size_t)dm * d.nslot + slot] = v;
}

// V_D on the G box: zero, then each half-space slot writes V_D(G) at n and
// conj V_D(G) at -n (each box position is written by at most one slot)
__global__ __launch_bounds__(256) void k_gpw_zero(double2 *__restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_double2(0.0, 0.0);
}

__global__ __launch_bounds__(256) void k_gpw_from_slots(const Dev d) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x, dm = blockIdx.y;
  if (slot >= d.nslot || d.slot_v[slot] == 0.0) return;
  const int K0 = 2 * d.gM[0] + 1, K1 = 2 * d.gM[1] + 1, K2 = 2 * d.gM[2] + 1;
  const int *n = d.slot_miller + 3 * (size_t)slot;
  const double2 vc = d.VDc[(size_t)dm * d.nslot + slot];  // conj V_D(G)
  double2 *g = d.grid_c + (size_t)dm * K0 * K1 * K2;
  g[((size_t)(n[2] + d.gM[2]) * K1 + (n[1] + d.gM[1])) * K0 + (n[0] + d.gM[0])] = make_double2(vc.x, -vc.y);
  g[((size_t)(-n[2] + d.gM[2]) * K1 + (-n[1] + d.gM[1])) * K0 + (-n[0] + d.gM[0])] = vc;
}

// J partials of the DD pairs: workgroup per (DD pair, chunk of 16 Cartesian
// elements, density); threads stride over the grid points of each image box in
// order, the 256 lanes' sums are added by a fixed tree
constexpr int kGpwChunk = 16;

__global__ __launch_bounds__(256) void k_gpw_integrate(const Dev d) {
  __shared__ double red[kGpwChunk][256];
  const int k = blockIdx.x, ec0 = blockIdx.y * kGpwChunk, dm = blockIdx.z;
  const int q = d.dd_q[k];
  const BlockRec b = d.blocks[d.dd_blk[k]];
  const int la = d.sh_l[b.sa], lb = d.sh_l[b.sb];
  const int nca = ncart(la), ncb = ncart(lb), nel = nca * ncb;
  if (ec0 >= nel) return;  // the whole workgroup: no element of this chunk
  const PairAux x = d.aux[q];
  const double *V = d.grid_r + (size_t)dm * d.gpts;
  int ex[kGpwChunk][3], eb[kGpwChunk][3];
#pragma unroll
  for (int u = 0; u < kGpwChunk; ++u) {
    const int e = min(ec0 + u, nel - 1);
    gpw_cart(la, e / ncb, ex[u][0], ex[u][1], ex[u][2]);
    gpw_cart(lb, e % ncb, eb[u][0], eb[u][1], eb[u][2]);
  }
  double acc[kGpwChunk];
#pragma unroll
  for (int u = 0; u < kGpwChunk; ++u) acc[u] = 0.0;
  const double rc2 = d.gP[4 * k + 3];
  for (int ent = d.gimg_off[k]; ent < d.gimg_off[k + 1]; ++ent) {
    const int *box = d.gimg_box + 6 * (size_t)ent;
    const int m0 = d.gimg[4 * ent + 1], m1 = d.gimg[4 * ent + 2], m2 = d.gimg[4 * ent + 3];
    double T[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) T[c] = d.lat[c * 3 + 0] * m0 + d.lat[c * 3 + 1] * m1 + d.lat[c * 3 + 2] * m2;
    const int n0 = box[1] - box[0] + 1, n1 = box[3] - box[2] + 1, n2 = box[5] - box[4] + 1;
    const int64_t nb = (int64_t)n0 * n1 * n2;
    for (int64_t u = threadIdx.x; u < nb; u += blockDim.x) {
      const int j0 = box[0] + (int)(u % n0), j1 = box[2] + (int)((u / n0) % n1), j2 = box[4] + (int)(u / ((int64_t)n0 * n1));
      double r[3], X[3], x2 = 0.0;
      gpw_point(d, j0, j1, j2, r);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        X[c] = r[c] - d.gP[4 * k + c] - T[c];
        x2 += X[c] * X[c];
      }
      if (x2 > rc2) continue;
      const double g = V[((size_t)j2 * d.gN[1] + j1) * d.gN[0] + j0] * exp(-x.p * x2);
      double pa[3][kMaxL + 1], pb[3][kMaxL + 1];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        pa[c][0] = pb[c][0] = 1.0;
#pragma unroll
        for (int i = 1; i <= kMaxL; ++i) {
          pa[c][i] = pa[c][i - 1] * (X[c] + x.xpa[c]);
          pb[c][i] = pb[c][i - 1] * (X[c] + x.xpb[c]);
        }
      }
#pragma unroll
      for (int v = 0; v < kGpwChunk; ++v) {
        double f = g;
#pragma unroll
        for (int c = 0; c < 3; ++c) f *= pa[c][ex[v][c]] * pb[c][eb[v][c]];
        acc[v] += f;
      }
    }
  }
#pragma unroll
  for (int v = 0; v < kGpwChunk; ++v) red[v][threadIdx.x] = acc[v];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
#pragma unroll
      for (int v = 0; v < kGpwChunk; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < kGpwChunk && ec0 + (int)threadIdx.x < nel) {
    const double w = gpw_pref(x) * d.vol / (double)d.gpts;
    d.gpw_part[((size_t)dm * d.ndd + k) * kGpwEl + ec0 + threadIdx.x] = w * red[threadIdx.x][0];
  }
}

// J(L) += the DD pairs' partials, each block's DD pairs (consecutive in the DD
// list) added in list order by the thread of its first pair
__global__ __launch_bounds__(256) void k_gpw_add(const Dev d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int dm = blockIdx.y;
  if (i >= (int64_t)d.ndd * kGpwEl) return;
  const int k = (int)(i / kGpwEl), e = (int)(i % kGpwEl);
  if (k > 0 && d.dd_blk[k - 1] == d.dd_blk[k]) return;
  const BlockRec b = d.blocks[d.dd_blk[k]];
  const int nel = ncart(d.sh_l[b.sa]) * ncart(d.sh_l[b.sb]);
  if (e >= nel) return;
  double s = 0.0;
  for (int kk = k; kk < d.ndd && d.dd_blk[kk] == d.dd_blk[k]; ++kk) s += d.gpw_part[((size_t)dm * d.ndd + kk) * kGpwEl + e];
  d.Jblk[(size_t)dm * d.nelem + b.eoff + e] += s;
}

#define PWDF_CHECK_LAUNCH_GPW()         \
  do {                                  \
    hipError_t e_ = hipGetLastError();  \
    if (e_ != hipSuccess) return e_;    \
  } while (0)

static hipError_t gpw_axis(const Dev &d, const double2 *in, const double *rin, double2 *out, double *rout, int d0,
                           int d1, int d2, int a, int nin, int sign, int forward, int ndm, hipStream_t st) {
  const int64_t n = (int64_t)d0 * d1 * d2;
  hipLaunchKernelGGL(k_gpw_axis, dim3((unsigned)((n + 255) / 256), ndm), dim3(256), 0, st, in, rin, out, rout, d0, d1,
                     d2, a, nin, d.gN[a], d.gM[a], sign, forward);
  PWDF_CHECK_LAUNCH_GPW();
  return hipSuccess;
}

hipError_t launch_gpw_rho(const Dev &d, int ndm, hipStream_t st) {
  const int N0 = d.gN[0], N1 = d.gN[1], N2 = d.gN[2];
  const int K0 = 2 * d.gM[0] + 1, K1 = 2 * d.gM[1] + 1, K2 = 2 * d.gM[2] + 1;
  const int ntiles = d.gtiles[0] * d.gtiles[1] * d.gtiles[2];
  hipLaunchKernelGGL(k_gpw_collocate, dim3((unsigned)d.ngitems, ndm), dim3(256), 0, st, d);
  PWDF_CHECK_LAUNCH_GPW();
  hipLaunchKernelGGL(k_gpw_collect, dim3((unsigned)ntiles, ndm), dim3(256), 0, st, d);
  PWDF_CHECK_LAUNCH_GPW();
  hipError_t e;
  if ((e = gpw_axis(d, nullptr, d.grid_r, d.grid_a, nullptr, K0, N1, N2, 0, N0, -1, 1, ndm, st)) != hipSuccess) return e;
  if ((e = gpw_axis(d, d.grid_a, nullptr, d.grid_b, nullptr, K0, K1, N2, 1, N1, -1, 1, ndm, st)) != hipSuccess) return e;
  if ((e = gpw_axis(d, d.grid_b, nullptr, d.grid_c, nullptr, K0, K1, K2, 2, N2, -1, 1, ndm, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_gpw_to_slots, dim3((unsigned)((d.nslot + 255) / 256), ndm), dim3(256), 0, st, d);
  PWDF_CHECK_LAUNCH_GPW();
  return hipSuccess;
}

hipError_t launch_gpw_j(const Dev &d, int ndm, hipStream_t st) {
  const int N0 = d.gN[0], N1 = d.gN[1], N2 = d.gN[2];
  const int K0 = 2 * d.gM[0] + 1, K1 = 2 * d.gM[1] + 1, K2 = 2 * d.gM[2] + 1;
  const int64_t nc = (int64_t)K0 * K1 * K2 * ndm;
  hipLaunchKernelGGL(k_gpw_zero, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, d.grid_c, nc);
  PWDF_CHECK_LAUNCH_GPW();
  hipLaunchKernelGGL(k_gpw_from_slots, dim3((unsigned)((d.nslot + 255) / 256), ndm), dim3(256), 0, st, d);
  PWDF_CHECK_LAUNCH_GPW();
  hipError_t e;
  if ((e = gpw_axis(d, d.grid_c, nullptr, d.grid_b, nullptr, K0, K1, N2, 2, K2, 1, 0, ndm, st)) != hipSuccess) return e;
  if ((e = gpw_axis(d, d.grid_b, nullptr, d.grid_a, nullptr, K0, N1, N2, 1, K1, 1, 0, ndm, st)) != hipSuccess) return e;
  if ((e = gpw_axis(d, d.grid_a, nullptr, nullptr, d.grid_r, N0, N1, N2, 0, K0, 1, 0, ndm, st)) != hipSuccess) return e;
  const int nchunks = (kGpwEl + kGpwChunk - 1) / kGpwChunk;
  hipLaunchKernelGGL(k_gpw_integrate, dim3((unsigned)d.ndd, nchunks, ndm), dim3(256), 0, st, d);
  PWDF_CHECK_LAUNCH_GPW();
  return hipSuccess;
}

hipError_t launch_gpw_add(const Dev &d, int ndm, hipStream_t st) {
  const int64_t n = (int64_t)d.ndd * kGpwEl;
  hipLaunchKernelGGL(k_gpw_add, dim3((unsigned)((n + 255) / 256), ndm), dim3(256), 0, st, d);
  PWDF_CHECK_LAUNCH_GPW();
  return hipSuccess;
}

}  // namespace pwdf
