// HIP kernels of the DD solver for gfx950 (CDNA4).
//
// Storage: every dense matrix is column-major and planar complex (real plane,
// then imaginary plane).  Complex products C += A B are split into four real
// MFMA products: Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br.
//
// Blocked LDL^T of a front with s fully-summed columns (pivot tiles of NB):
//   tile k:  P_k A_kk P_k^T = L_kk D_k L_kk^T   (restricted Bunch-Kaufman:
//            the pivot search never leaves the NB x NB diagonal tile)
//            -> the strict lower triangle of the diagonal tile receives
//               L_kk^-1, D_k^-1 goes to the side arrays
//   W   = A_21 P_k^T L_kk^-T        (= L_21 D_k, kept in the W scratch)
//   L21 = W D_k^-1                  (stored in place of A_21)
//   A22 -= L21 W^T                  (lower tiles only)
// Row permutations of earlier column blocks are not applied ("lazy"): the
// substitutions apply P_k when they reach tile k, which is equivalent.
#include <hip/hip_runtime.h>

#include <cstdio>

#include "dd_internal.h"
#include "kernels.h"

namespace dd {

struct cd {
  double re, im;
};

template <typename T>
struct KP {
  const FrontDev *F;
  const Item *items;
  const int32_t *vars;
  const int32_t *cfront;
  const int64_t *crmap;
  const int32_t *rmap;
  const SPair *spairs;
  const AuxItem *aux;
  const int32_t *gpos;
  const int32_t *gsign;
  const MultRef *mrefs;
  const GamRef *grefs;
  const int32_t *hmult;
  const int32_t *hsign;
  const int32_t *rowgam;
  const int64_t *csrp;
  const int32_t *csrc;
  const Item *gemv;
  T *num;
  cd *dinv;
  cd *doff;
  int32_t *pdel;
  int32_t *perm;
  const cd *vals;
  int *status;
  double *r64;
  int64_t vf, vx, vd, vl, vc, part;
  int64_t n_torn, n_mult;
  int32_t mr;
};

// ---------------------------------------------------------------------------
// MFMA helpers
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
template <typename T>
struct V4;
template <>
struct V4<double> {
  typedef v4d t;
};
template <>
struct V4<float> {
  typedef v4f t;
};

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int TK = 16;
constexpr int LP = GT + 4;

template <typename T>
struct GemmSmem {
  T a[2][TK][LP];
  T b[2][TK][LP];
};

// Accumulates a GT x GT complex tile P = sum_k A(m,k) B(c,k) over k in
// [kbeg, kend).  fa(m, k, re, im) / fb(c, k, re, im) return operand values
// (and must leave zeros outside their valid range).  AK / BK select the
// thread mapping of the loads: true when the operand is contiguous along k.
// The next K chunk is fetched into registers while the current one is
// multiplied.  Wave w owns rows 32*(w/2) + [0,32) and columns 32*(w%2) +
// [0,32) as 2x2 MFMA 16x16 blocks.  The MFMA computes the transposed block
// (first operand from B, second from A) so that the 16 lanes of a result row
// run along m, the contiguous dimension of the column-major tiles; out_row /
// out_col give the element positions.
template <typename T, bool AK, bool BK, class FA, class FB>
__device__ __forceinline__ void gemm_tile(GemmSmem<T> &sm, int kbeg, int kend, FA fa, FB fb,
                                          typename V4<T>::t (&cr)[2][2], typename V4<T>::t (&ci)[2][2]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      cr[x][y] = typename V4<T>::t{0, 0, 0, 0};
      ci[x][y] = typename V4<T>::t{0, 0, 0, 0};
    }
  T ra[2][4], rb[2][4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int rep = 0; rep < 4; ++rep) {
      const int m = AK ? (tid >> 4) + 16 * rep : (tid & 63);
      const int k = AK ? (tid & 15) : (tid >> 6) + 4 * rep;
      T re = 0, im = 0;
      if (k0 + k < kend) fa(m, k0 + k, re, im);
      ra[0][rep] = re;
      ra[1][rep] = im;
    }
#pragma unroll
    for (int rep = 0; rep < 4; ++rep) {
      const int m = BK ? (tid >> 4) + 16 * rep : (tid & 63);
      const int k = BK ? (tid & 15) : (tid >> 6) + 4 * rep;
      T re = 0, im = 0;
      if (k0 + k < kend) fb(m, k0 + k, re, im);
      rb[0][rep] = re;
      rb[1][rep] = im;
    }
  };
  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += TK) {
    __syncthreads();
#pragma unroll
    for (int rep = 0; rep < 4; ++rep) {
      const int ma = AK ? (tid >> 4) + 16 * rep : (tid & 63);
      const int ka = AK ? (tid & 15) : (tid >> 6) + 4 * rep;
      sm.a[0][ka][ma] = ra[0][rep];
      sm.a[1][ka][ma] = ra[1][rep];
      const int mb = BK ? (tid >> 4) + 16 * rep : (tid & 63);
      const int kb = BK ? (tid & 15) : (tid >> 6) + 4 * rep;
      sm.b[0][kb][mb] = rb[0][rep];
      sm.b[1][kb][mb] = rb[1][rep];
    }
    __syncthreads();
    if (k0 + TK < kend) fetch(k0 + TK);
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const int kr = kk + (lane >> 4);
      T ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        ar[x] = sm.a[0][kr][wr * 32 + x * 16 + (lane & 15)];
        ai[x] = sm.a[1][kr][wr * 32 + x * 16 + (lane & 15)];
        br[x] = sm.b[0][kr][wc * 32 + x * 16 + (lane & 15)];
        bi[x] = sm.b[1][kr][wc * 32 + x * 16 + (lane & 15)];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          cr[x][y] = mfma16(br[y], ar[x], cr[x][y]);
          cr[x][y] = mfma16(-bi[y], ai[x], cr[x][y]);
          ci[x][y] = mfma16(bi[y], ar[x], ci[x][y]);
          ci[x][y] = mfma16(br[y], ai[x], ci[x][y]);
        }
    }
  }
}

// Position of element i of result block (x, y): row (the m index) and
// column (the c index) inside the GT x GT tile.  The MFMA result row index is
// 4*(lane/16) + i for the FP32 instruction and lane/16 + 4*i for the FP64 one;
// its column is lane%16.
__device__ __forceinline__ int out_row(int x) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  return (w >> 1) * 32 + x * 16 + (lane & 15);
}
template <typename T>
__device__ __forceinline__ int out_col(int y, int i) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (sizeof(T) == 8) return (w & 1) * 32 + y * 16 + (lane >> 4) + 4 * i;
  return (w & 1) * 32 + y * 16 + (lane >> 4) * 4 + i;
}

__device__ __forceinline__ double cabs1(double r, double i) { return fabs(r) + fabs(i); }

// ---------------------------------------------------------------------------
// assembly: pull extend-add.  Workgroup item (f, c0, r0) assigns the
// lower-triangle entries of rows [r0, r0+256) x columns [c0, c0+64) of front
// f: the sum of the children's update-block entries mapped there (zero where
// no child contributes).  Children are taken in groups of 8; a thread keeps
// the children's row-map entries of its row in registers, the column maps of
// the block sit in LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_asm(KP<T> p, int64_t first) {
  __shared__ int rmc[8][64];
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, c0 = it.k, r = it.i + threadIdx.x;
  const int cend = min(c0 + 64, n);
  T *re = p.num + f.off;
  T *im = re + (int64_t)n * n;
  for (int g0 = 0; g0 < max(f.nchild, 1); g0 += 8) {
    const int ng = min(8, f.nchild - g0);
    __syncthreads();
    for (int e = threadIdx.x; e < 8 * 64; e += 256) {
      const int ch = e / 64, c = c0 + (e % 64);
      rmc[ch][e % 64] = (ch < ng && c < n) ? p.rmap[p.crmap[f.child + g0 + ch] + c] : -1;
    }
    __syncthreads();
    if (r >= n) continue;
    int rr[8];
    int64_t coff[8], cn[8], cplane[8];
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) {
      rr[ch] = -1;
      coff[ch] = cn[ch] = cplane[ch] = 0;
      if (ch < ng) {
        rr[ch] = p.rmap[p.crmap[f.child + g0 + ch] + r];
        const FrontDev &cf = p.F[p.cfront[f.child + g0 + ch]];
        cn[ch] = cf.n;
        cplane[ch] = (int64_t)cf.n * cf.n;
        coff[ch] = cf.off + cf.s + (int64_t)cf.s * cf.n;   // origin of the update block
      }
    }
    for (int c = c0; c < cend && c <= r; ++c) {
      T vr = 0, vi = 0;
#pragma unroll
      for (int ch = 0; ch < 8; ++ch) {
        const int rc = rmc[ch][c - c0];
        if (rr[ch] >= 0 && rc >= 0) {
          const int64_t o = coff[ch] + rr[ch] + rc * cn[ch];
          vr += p.num[o];
          vi += p.num[o + cplane[ch]];
        }
      }
      const int64_t o = r + (int64_t)c * n;
      if (g0 == 0) {
        re[o] = vr;
        im[o] = vi;
      } else {
        re[o] += vr;
        im[o] += vi;
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_scat(KP<T> p, int64_t first) {
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  T *re = p.num + f.off;
  T *im = re + (int64_t)f.n * f.n;
  for (int e = threadIdx.x; e < it.i; e += 256) {
    const SPair sp = p.spairs[(int64_t)it.k + e];
    const cd v = p.vals[sp.src];
    re[sp.pos] += (T)v.re;
    im[sp.pos] += (T)v.im;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_auxg(KP<T> p, int64_t first) {
  const Item it = p.items[first + blockIdx.x];
  const AuxItem a = p.aux[it.f];
  const FrontDev f = p.F[a.f];
  T *re = p.num + f.off;
  T *im = re + (int64_t)f.n * f.n;
  const int total = a.na * a.nb;
  for (int e = threadIdx.x; e < total; e += 256) {
    const int j = e % a.nb, i = e / a.nb;
    if (a.same && j < i) continue;
    T sr = 0, si = 0;
    for (int t = 0; t < a.ndom; ++t) {
      const int64_t ga = p.gpos[a.ga[t] + i], gb = p.gpos[a.gb[t] + j];
      const int sg = p.gsign[a.ga[t] + i] * p.gsign[a.gb[t] + j];
      const int64_t g = a.g[t];
      const T *X = p.num + a.xoff[t];
      const T xr = X[gb + ga * g], xi = X[g * g + gb + ga * g];
      sr += sg > 0 ? xr : -xr;
      si += sg > 0 ? xi : -xi;
    }
    const int64_t o = (a.pb + j) + (int64_t)(a.pa + i) * f.n;
    re[o] += sr;
    im[o] += si;
  }
}

// ---------------------------------------------------------------------------
// pivot tile: restricted Bunch-Kaufman LDL^T of the NB x NB diagonal tile, in
// FP64 in LDS (both triangles kept), with L^-1 formed alongside.
__device__ __forceinline__ void wave_argmax(double &v, int &idx) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const int oi = __shfl_xor(idx, off);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_panel(KP<T> p, int64_t first) {
  __shared__ double Ar[NB][NB + 1], Ai[NB][NB + 1];
  __shared__ double Yr[NB][NB + 1], Yi[NB][NB + 1];
  __shared__ double v0r[NB], v0i[NB], v1r[NB], v1i[NB], l0r[NB], l0i[NB], l1r[NB], l1i[NB];
  __shared__ double dvr[NB], dvi[NB], dor[NB], doi[NB];
  __shared__ int pdl[NB], pv[NB];
  __shared__ int s_kind, s_piv, s_pert;
  __shared__ double s_amax;

  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int k = it.k, n = f.n, b = min(NB, f.s - k), tid = threadIdx.x;
  T *fr = p.num + f.off;
  T *fi = fr + (int64_t)n * n;
  constexpr double ALPHA = 0.6403882032022076;   // (1 + sqrt(17)) / 8

  double amax = 0;
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e % NB, j = e / NB;
    if (i < b && j < b && i >= j) {
      const int64_t o = (k + i) + (int64_t)(k + j) * n;
      const double xr = (double)fr[o], xi = (double)fi[o];
      Ar[i][j] = xr;
      Ai[i][j] = xi;
      Ar[j][i] = xr;
      Ai[j][i] = xi;
      amax = fmax(amax, cabs1(xr, xi));
    }
    if (i < NB && j < NB) {
      Yr[i][j] = (i == j) ? 1.0 : 0.0;
      Yi[i][j] = 0.0;
    }
  }
  if (tid < NB) pv[tid] = tid;
  // block max for the perturbation scale
  {
    __shared__ double red[4];
    amax = wave_max(amax);
    if ((tid & 63) == 0) red[tid >> 6] = amax;
    __syncthreads();
    if (tid == 0) {
      s_amax = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
      s_pert = 0;
    }
    __syncthreads();
  }
  const double tau = s_amax > 0 ? 1e-12 * s_amax : 1.0;

  int j = 0;
  while (j < b) {
    if (tid < 64) {
      const int i = tid;
      const double absakk = cabs1(Ar[j][j], Ai[j][j]);
      double cv = (i > j && i < b) ? cabs1(Ar[i][j], Ai[i][j]) : -1.0;
      int imax = i;
      wave_argmax(cv, imax);
      const double colmax = cv;
      int kind = 1, piv = j;
      if (colmax > 0.0 && absakk < ALPHA * colmax) {
        double rv = (i >= j && i < b && i != imax) ? cabs1(Ar[imax][i], Ai[imax][i]) : -1.0;
        const double rowmax = wave_max(rv);
        if (absakk * rowmax >= ALPHA * colmax * colmax) {
          kind = 1;
          piv = j;
        } else if (cabs1(Ar[imax][imax], Ai[imax][imax]) >= ALPHA * rowmax) {
          kind = 1;
          piv = imax;
        } else {
          kind = 2;
          piv = imax;
        }
      }
      if (tid == 0) {
        s_kind = kind;
        s_piv = piv;
      }
    }
    __syncthreads();
    const int kind = s_kind, piv = s_piv;
    const int q = (kind == 1) ? j : j + 1;
    if (piv != q) {
      for (int c = tid; c < b; c += 256) {
        double t = Ar[q][c]; Ar[q][c] = Ar[piv][c]; Ar[piv][c] = t;
        t = Ai[q][c]; Ai[q][c] = Ai[piv][c]; Ai[piv][c] = t;
      }
      for (int c = tid; c < j; c += 256) {
        double t = Yr[q][c]; Yr[q][c] = Yr[piv][c]; Yr[piv][c] = t;
        t = Yi[q][c]; Yi[q][c] = Yi[piv][c]; Yi[piv][c] = t;
      }
      if (tid == 0) {
        int t = pv[q]; pv[q] = pv[piv]; pv[piv] = t;
      }
      __syncthreads();
      for (int r = j + tid; r < b; r += 256) {
        double t = Ar[r][q]; Ar[r][q] = Ar[r][piv]; Ar[r][piv] = t;
        t = Ai[r][q]; Ai[r][q] = Ai[r][piv]; Ai[r][piv] = t;
      }
      __syncthreads();
    }
    if (kind == 1) {
      double dr = Ar[j][j], di = Ai[j][j];
      if (dr == 0.0 && di == 0.0) {
        dr = tau;
        if (tid == 0) s_pert++;
      }
      const double den = dr * dr + di * di;
      const double ir = dr / den, ii = -di / den;
      for (int i = j + 1 + tid; i < b; i += 256) {
        const double vr = Ar[i][j], vi = Ai[i][j];
        v0r[i] = vr;
        v0i[i] = vi;
        l0r[i] = vr * ir - vi * ii;
        l0i[i] = vr * ii + vi * ir;
      }
      if (tid == 0) {
        dvr[j] = ir; dvi[j] = ii; dor[j] = 0; doi[j] = 0; pdl[j] = 0;
      }
      __syncthreads();
      const int m = b - j - 1;
      for (int e = tid; e < m * m; e += 256) {
        const int i = j + 1 + e % m, c = j + 1 + e / m;
        Ar[i][c] -= v0r[i] * l0r[c] - v0i[i] * l0i[c];
        Ai[i][c] -= v0r[i] * l0i[c] + v0i[i] * l0r[c];
      }
      for (int e = tid; e < m * (j + 1); e += 256) {
        const int i = j + 1 + e % m, c = e / m;
        const double yr = Yr[j][c], yi = Yi[j][c];
        Yr[i][c] -= l0r[i] * yr - l0i[i] * yi;
        Yi[i][c] -= l0r[i] * yi + l0i[i] * yr;
      }
      __syncthreads();
      j += 1;
    } else {
      double ar = Ar[j][j], ai = Ai[j][j], cr = Ar[j + 1][j], ci = Ai[j + 1][j];
      double er = Ar[j + 1][j + 1], ei = Ai[j + 1][j + 1];
      double detr = (ar * er - ai * ei) - (cr * cr - ci * ci);
      double deti = (ar * ei + ai * er) - 2.0 * cr * ci;
      if (detr == 0.0 && deti == 0.0) {
        ar += tau;
        er += tau;
        detr = (ar * er - ai * ei) - (cr * cr - ci * ci);
        deti = (ar * ei + ai * er) - 2.0 * cr * ci;
        if (tid == 0) s_pert++;
      }
      const double den = detr * detr + deti * deti;
      const double idr = detr / den, idi = -deti / den;   // 1/det
      // D^-1 = [[e, -c], [-c, a]] / det
      const double d00r = er * idr - ei * idi, d00i = er * idi + ei * idr;
      const double d11r = ar * idr - ai * idi, d11i = ar * idi + ai * idr;
      const double d01r = -(cr * idr - ci * idi), d01i = -(cr * idi + ci * idr);
      for (int i = j + 2 + tid; i < b; i += 256) {
        const double xr = Ar[i][j], xi = Ai[i][j], yr = Ar[i][j + 1], yi = Ai[i][j + 1];
        v0r[i] = xr; v0i[i] = xi; v1r[i] = yr; v1i[i] = yi;
        l0r[i] = (xr * d00r - xi * d00i) + (yr * d01r - yi * d01i);
        l0i[i] = (xr * d00i + xi * d00r) + (yr * d01i + yi * d01r);
        l1r[i] = (xr * d01r - xi * d01i) + (yr * d11r - yi * d11i);
        l1i[i] = (xr * d01i + xi * d01r) + (yr * d11i + yi * d11r);
      }
      if (tid == 0) {
        dvr[j] = d00r; dvi[j] = d00i; dvr[j + 1] = d11r; dvi[j + 1] = d11i;
        dor[j] = d01r; doi[j] = d01i; dor[j + 1] = d01r; doi[j + 1] = d01i;
        pdl[j] = 1; pdl[j + 1] = -1;
      }
      __syncthreads();
      const int m = b - j - 2;
      for (int e = tid; e < m * m; e += 256) {
        const int i = j + 2 + e % m, c = j + 2 + e / m;
        Ar[i][c] -= (v0r[i] * l0r[c] - v0i[i] * l0i[c]) + (v1r[i] * l1r[c] - v1i[i] * l1i[c]);
        Ai[i][c] -= (v0r[i] * l0i[c] + v0i[i] * l0r[c]) + (v1r[i] * l1i[c] + v1i[i] * l1r[c]);
      }
      for (int e = tid; e < m * (j + 2); e += 256) {
        const int i = j + 2 + e % m, c = e / m;
        const double y0r = Yr[j][c], y0i = Yi[j][c], y1r = Yr[j + 1][c], y1i = Yi[j + 1][c];
        Yr[i][c] -= (l0r[i] * y0r - l0i[i] * y0i) + (l1r[i] * y1r - l1i[i] * y1i);
        Yi[i][c] -= (l0r[i] * y0i + l0i[i] * y0r) + (l1r[i] * y1i + l1i[i] * y1r);
      }
      __syncthreads();
      j += 2;
    }
  }
  // write L^-1 into the strict lower triangle of the diagonal tile
  for (int e = tid; e < b * b; e += 256) {
    const int i = e % b, c = e / b;
    if (i > c) {
      const int64_t o = (k + i) + (int64_t)(k + c) * n;
      fr[o] = (T)Yr[i][c];
      fi[o] = (T)Yi[i][c];
    }
  }
  bool bad = false;
  for (int a = tid; a < b; a += 256) {
    const int64_t s = f.soff + k + a;
    p.dinv[s] = cd{dvr[a], dvi[a]};
    p.doff[s] = cd{dor[a], doi[a]};
    p.pdel[s] = pdl[a];
    p.perm[s] = pv[a];
    if (!isfinite(dvr[a]) || !isfinite(dvi[a])) bad = true;
  }
  if (bad) atomicOr(p.status + 1, 1);
  if (tid == 0 && s_pert) atomicAdd(p.status, s_pert);
}

// W = A21 P^T L11^-T (rows r0..r0+GT), L21 = W D^-1
template <typename T>
__global__ __launch_bounds__(256) void k_trsm(KP<T> p, int64_t first) {
  __shared__ GemmSmem<T> sm;
  __shared__ T wr[GT][GT + 1], wi[GT][GT + 1];
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int k = it.k, r0 = it.i, n = f.n, b = min(NB, f.s - k);
  T *fr = p.num + f.off;
  T *fi = fr + (int64_t)n * n;
  const int32_t *pm = p.perm + f.soff + k;
  auto fa = [&](int m, int kk, T &re, T &im) {
    const int r = r0 + m;
    if (r < n && kk < b) {
      const int64_t o = r + (int64_t)(k + pm[kk]) * n;
      re = fr[o];
      im = fi[o];
    }
  };
  auto fb = [&](int c, int kk, T &re, T &im) {
    if (c < b && kk <= c) {
      if (kk == c) {
        re = 1;
        im = 0;
      } else {
        const int64_t o = (k + c) + (int64_t)(k + kk) * n;
        re = fr[o];
        im = fi[o];
      }
    }
  };
  typename V4<T>::t cr[2][2], ci[2][2];
  gemm_tile<T, false, false>(sm, 0, b, fa, fb, cr, ci);
  T *Wr = p.num + f.woff;
  T *Wi = Wr + (int64_t)n * f.wcols;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = out_row(x), c = out_col<T>(y, i);
        wr[m][c] = cr[x][y][i];
        wi[m][c] = ci[x][y][i];
        if (r0 + m < n && c < b) {
          Wr[(r0 + m) + (int64_t)(it.j + c) * n] = cr[x][y][i];
          Wi[(r0 + m) + (int64_t)(it.j + c) * n] = ci[x][y][i];
        }
      }
  __syncthreads();
  for (int e = threadIdx.x; e < GT * b; e += 256) {
    const int m = e % GT, c = e / GT, r = r0 + m;
    if (r >= n) continue;
    const int64_t s = f.soff + k + c;
    const cd d = p.dinv[s];
    double xr = (double)wr[m][c] * d.re - (double)wi[m][c] * d.im;
    double xi = (double)wr[m][c] * d.im + (double)wi[m][c] * d.re;
    const int pd = p.pdel[s];
    if (pd) {
      const cd o = p.doff[s];
      const double yr = (double)wr[m][c + pd], yi = (double)wi[m][c + pd];
      xr += yr * o.re - yi * o.im;
      xi += yr * o.im + yi * o.re;
    }
    fr[r + (int64_t)(k + c) * n] = (T)xr;
    fi[r + (int64_t)(k + c) * n] = (T)xi;
  }
}

// Update of the trailing part by the factored columns [k, kend) of the current
// outer block: C(r0.., q0..) -= L21(r0.., k..kend) W(q0.., 0..kend-k)^T.
// Trailing update (q0 >= block end): lower tiles of the trailing matrix,
// kend = min(k + KBLK, s).  Column update (q0 < block end): the pivot tile
// column starting at q0 receives the block's earlier tiles, kend = q0.
template <typename T>
__global__ __launch_bounds__(256) void k_syrk(KP<T> p, int64_t first) {
  __shared__ GemmSmem<T> sm;
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int k = it.k, r0 = it.i, q0 = it.j, n = f.n;
  const int bend = min(k + KBLK, f.s);
  const bool colupd = q0 < bend;
  const int kend = colupd ? q0 : bend;
  const int qend = colupd ? min(q0 + NB, f.s) : n;
  T *fr = p.num + f.off;
  T *fi = fr + (int64_t)n * n;
  const T *Wr = p.num + f.woff;
  const T *Wi = Wr + (int64_t)n * f.wcols;
  auto fa = [&](int m, int kk, T &re, T &im) {
    const int r = r0 + m;
    if (r < n) {
      const int64_t o = r + (int64_t)kk * n;
      re = fr[o];
      im = fi[o];
    }
  };
  auto fb = [&](int c, int kk, T &re, T &im) {
    const int q = q0 + c;
    if (q < qend) {
      const int64_t o = q + (int64_t)(kk - k) * n;
      re = Wr[o];
      im = Wi[o];
    }
  };
  typename V4<T>::t cr[2][2], ci[2][2];
  gemm_tile<T, false, false>(sm, k, kend, fa, fb, cr, ci);
  const bool diag = (r0 == q0);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = out_row(x), c = out_col<T>(y, i);
        const int r = r0 + m, q = q0 + c;
        if (r < n && q < qend && (!diag || m >= c)) {
          const int64_t o = r + (int64_t)q * n;
          fr[o] -= cr[x][y][i];
          fi[o] -= ci[x][y][i];
        }
      }
}

// ---------------------------------------------------------------------------
// interface root inverse X = S^-1 from P S P^T = L D L^T (lazy tile perms):
// Z = L_true^-1 column block by column block (descending), then
// X = P^T Z^T D^-1 Z P.  Diagonal tiles already hold Z_kk = L_kk^-1.
template <typename T>
__device__ __forceinline__ void zval(const T *fr, const T *fi, int n, int r, int c, T &re, T &im) {
  // Z(r, c) of a unit lower triangular matrix stored in the lower triangle
  if (r > c) {
    const int64_t o = r + (int64_t)c * n;
    re = fr[o];
    im = fi[o];
  } else if (r == c) {
    re = 1;
    im = 0;
  }
}

// Recursive inverse of the fully-summed block: for a tile range split at m0
// whose two halves already hold Z, with L_true = P L_stored (lazy tile perms):
//   T1  = L_true(second half rows, first half cols) Z11   -> upper triangle (transposed)
//   Z21 = -Z22 T1                                         -> lower triangle
// Item (f, m0, r0, c0): output tile rows [r0, r0+64), columns [c0, c0+64).
template <typename T>
__global__ __launch_bounds__(256) void k_zrec1(KP<T> p, int64_t first) {
  __shared__ GemmSmem<T> sm;
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int m0 = it.k, r0 = it.i, c0 = it.j, n = f.n, s = f.s;
  T *fr = p.num + f.off;
  T *fi = fr + (int64_t)n * n;
  const int32_t *pm = p.perm + f.soff;
  auto fa = [&](int m, int kk, T &re, T &im) {
    const int r = r0 + m;
    if (r < s) {
      const int rs = (r / NB) * NB + pm[r];
      const int64_t o = rs + (int64_t)kk * n;
      re = fr[o];
      im = fi[o];
    }
  };
  auto fb = [&](int c, int kk, T &re, T &im) {   // Z(kk, c0 + c)
    zval(fr, fi, n, kk, c0 + c, re, im);
  };
  typename V4<T>::t cr[2][2], ci[2][2];
  gemm_tile<T, false, true>(sm, c0, m0, fa, fb, cr, ci);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = out_row(x), c = out_col<T>(y, i);
        if (r0 + m < s && c0 + c < m0) {
          const int64_t o = (c0 + c) + (int64_t)(r0 + m) * n;
          fr[o] = cr[x][y][i];
          fi[o] = ci[x][y][i];
        }
      }
}

template <typename T>
__global__ __launch_bounds__(256) void k_zrec2(KP<T> p, int64_t first) {
  __shared__ GemmSmem<T> sm;
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int m0 = it.k, r0 = it.i, c0 = it.j, n = f.n, s = f.s;
  T *fr = p.num + f.off;
  T *fi = fr + (int64_t)n * n;
  auto fa = [&](int m, int kk, T &re, T &im) {   // Z(r0 + m, kk)
    const int r = r0 + m;
    if (r < s) zval(fr, fi, n, r, kk, re, im);
  };
  auto fb = [&](int c, int kk, T &re, T &im) {   // T1(kk, c0 + c), stored at (c0 + c, kk)
    if (c0 + c < m0) {
      const int64_t o = (c0 + c) + (int64_t)kk * n;
      re = fr[o];
      im = fi[o];
    }
  };
  typename V4<T>::t cr[2][2], ci[2][2];
  gemm_tile<T, false, false>(sm, m0, min(r0 + GT, s), fa, fb, cr, ci);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = out_row(x), c = out_col<T>(y, i);
        if (r0 + m < s && c0 + c < m0) {
          const int64_t o = (r0 + m) + (int64_t)(c0 + c) * n;
          fr[o] = -cr[x][y][i];
          fi[o] = -ci[x][y][i];
        }
      }
}

// X(P a, P c) = sum_r Z(r, a) (D^-1 Z)(r, c), lower tiles, written to both triangles
template <typename T>
__global__ __launch_bounds__(256) void k_invsyrk(KP<T> p, int64_t first) {
  __shared__ GemmSmem<T> sm;
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int a0 = it.i, c0 = it.j, n = f.n;
  const T *fr = p.num + f.off;
  const T *fi = fr + (int64_t)n * n;
  const cd *dv = p.dinv + f.soff;
  const cd *dof = p.doff + f.soff;
  const int32_t *pd = p.pdel + f.soff;
  const int32_t *pm = p.perm + f.soff;
  auto fa = [&](int m, int kk, T &re, T &im) {
    const int a = a0 + m;
    if (a < n) zval(fr, fi, n, kk, a, re, im);
  };
  auto fb = [&](int c, int kk, T &re, T &im) {
    const int cc = c0 + c;
    if (cc >= n) return;
    T zr = 0, zi = 0;
    zval(fr, fi, n, kk, cc, zr, zi);
    const cd d = dv[kk];
    double xr = d.re * (double)zr - d.im * (double)zi;
    double xi = d.re * (double)zi + d.im * (double)zr;
    const int q = pd[kk];
    if (q) {
      T wr = 0, wi = 0;
      zval(fr, fi, n, kk + q, cc, wr, wi);
      const cd o = dof[kk];
      xr += o.re * (double)wr - o.im * (double)wi;
      xi += o.re * (double)wi + o.im * (double)wr;
    }
    re = (T)xr;
    im = (T)xi;
  };
  typename V4<T>::t cr[2][2], ci[2][2];
  gemm_tile<T, true, true>(sm, a0, n, fa, fb, cr, ci);
  T *Xr = p.num + f.xoff;
  T *Xi = Xr + (int64_t)n * n;
  const bool diag = (a0 == c0);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = out_row(x), c = out_col<T>(y, i);
        const int a = a0 + m, cc = c0 + c;
        if (a < n && cc < n && (!diag || m >= c)) {
          const int pa = (a / NB) * NB + pm[a], pc = (cc / NB) * NB + pm[cc];
          Xr[pa + (int64_t)pc * n] = cr[x][y][i];
          Xi[pa + (int64_t)pc * n] = ci[x][y][i];
          Xr[pc + (int64_t)pa * n] = cr[x][y][i];
          Xi[pc + (int64_t)pa * n] = ci[x][y][i];
        }
      }
}

// ---------------------------------------------------------------------------
// multi-RHS substitutions (front vectors v: n x mr planar, ld n)
template <typename T>
__global__ __launch_bounds__(256) void k_finit(KP<T> p, int64_t first, int nrhs) {
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, s = f.s;
  const int64_t mr = p.mr;
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)n * mr;
  const bool aux = f.kind == FK_AUX;
  const int64_t ld = aux ? p.n_mult : p.n_torn;
  const T *sr = p.num + (aux ? p.vd : p.vf);
  const T *si = sr + ld * mr;
  for (int e = threadIdx.x; e < n * nrhs; e += 256) {
    const int r = e % n, j = e / n;
    T xr = 0, xi = 0;
    if (r < s) {
      const int64_t row = f.vbase + p.vars[f.idx + r] + (int64_t)j * ld;
      xr = sr[row];
      xi = si[row];
    }
    for (int ch = 0; ch < f.nchild; ++ch) {
      const int rr = p.rmap[p.crmap[f.child + ch] + r];
      if (rr < 0) continue;
      const FrontDev &cf = p.F[p.cfront[f.child + ch]];
      const int64_t o = cf.voff + cf.s + rr + (int64_t)j * cf.n;
      xr += p.num[o];
      xi += p.num[o + (int64_t)cf.n * mr];
    }
    vr[r + (int64_t)j * n] = xr;
    vi[r + (int64_t)j * n] = xi;
  }
}

// Loads the strict lower triangle of the diagonal tile (L_kk^-1) into LDS.
template <typename T>
__device__ __forceinline__ void load_ytile(T (&yr)[NB][NB + 1], T (&yi)[NB][NB + 1], const T *fr, const T *fi,
                                           int n, int k, int b) {
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int a = e % NB, c = e / NB;
    T vr = 0, vi = 0;
    if (a < b && c < a) {
      const int64_t o = (k + a) + (int64_t)(k + c) * n;
      vr = fr[o];
      vi = fi[o];
    }
    yr[a][c] = vr;
    yi[a][c] = vi;
  }
}

// y_k = L_kk^-1 P_k v_k for columns [j0, j0+nj) of the front vector v (ld n);
// y is also left in (sr, si).
template <typename T>
__device__ __forceinline__ void tile_forward(T (&sr)[NB][65], T (&si)[NB][65], const T (&yr)[NB][NB + 1],
                                             const T (&yi)[NB][NB + 1], T *vr, T *vi, int n, int k, int b,
                                             const int32_t *pm, int j0, int nj) {
  const int tid = threadIdx.x;
  for (int e = tid; e < b * nj; e += 256) {
    const int a = e % b, j = e / b;
    const int64_t o = k + pm[a] + (int64_t)(j0 + j) * n;
    sr[a][j] = vr[o];
    si[a][j] = vi[o];
  }
  __syncthreads();
  T ur[16], ui[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q;
    ur[q] = ui[q] = 0;
    if (e < b * nj) {
      const int a = e % b, j = e / b;
      T xr = sr[a][j], xi = si[a][j];
      for (int c = 0; c < a; ++c) {
        const T lr = yr[a][c], li = yi[a][c];
        xr += lr * sr[c][j] - li * si[c][j];
        xi += lr * si[c][j] + li * sr[c][j];
      }
      ur[q] = xr;
      ui[q] = xi;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q;
    if (e < b * nj) {
      const int a = e % b, j = e / b;
      sr[a][j] = ur[q];
      si[a][j] = ui[q];
      vr[k + a + (int64_t)(j0 + j) * n] = ur[q];
      vi[k + a + (int64_t)(j0 + j) * n] = ui[q];
    }
  }
  __syncthreads();
}

// v(r, j0..j0+nj) -= L(r, k..k+b) y for one row r (y in sr/si)
template <typename T>
__device__ __forceinline__ void row_update(const T (&sr)[NB][65], const T (&si)[NB][65], const T *fr, const T *fi,
                                           T *vr, T *vi, int n, int k, int b, int r, int j0, int nj) {
  for (int jj = 0; jj < nj; jj += 8) {
    T ar[8], ai[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) ar[q] = ai[q] = 0;
    int c = 0;
    for (; c + 4 <= b; c += 4) {
      T lr[4], li[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t o = r + (int64_t)(k + c + u) * n;
        lr[u] = fr[o];
        li[u] = fi[o];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          ar[q] += lr[u] * sr[c + u][jj + q] - li[u] * si[c + u][jj + q];
          ai[q] += lr[u] * si[c + u][jj + q] + li[u] * sr[c + u][jj + q];
        }
    }
    for (; c < b; ++c) {
      const int64_t o = r + (int64_t)(k + c) * n;
      const T lr = fr[o], li = fi[o];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        ar[q] += lr * sr[c][jj + q] - li * si[c][jj + q];
        ai[q] += lr * si[c][jj + q] + li * sr[c][jj + q];
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (jj + q < nj) {
        const int64_t o = r + (int64_t)(j0 + jj + q) * n;
        vr[o] -= ar[q];
        vi[o] -= ai[q];
      }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fdiag(KP<T> p, int64_t first, int nrhs) {
  __shared__ T sr[NB][65], si[NB][65];
  __shared__ T yr[NB][NB + 1], yi[NB][NB + 1];
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, k = it.k, b = min(NB, f.s - k);
  const int64_t mr = p.mr;
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)n * mr;
  const T *fr = p.num + f.off;
  const T *fi = fr + (int64_t)n * n;
  load_ytile(yr, yi, fr, fi, n, k, b);
  for (int j0 = 0; j0 < nrhs; j0 += 64) {
    const int nj = min(64, nrhs - j0);
    tile_forward(sr, si, yr, yi, vr, vi, n, k, b, p.perm + f.soff + k, j0, nj);
  }
}

// v(rows r0..r0+255, r >= k+b) -= L21(:, tile k) y_k
template <typename T>
__global__ __launch_bounds__(256) void k_fupd(KP<T> p, int64_t first, int nrhs) {
  __shared__ T sr[NB][65], si[NB][65];
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, k = it.k, b = min(NB, f.s - k);
  const int64_t mr = p.mr;
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)n * mr;
  const T *fr = p.num + f.off;
  const T *fi = fr + (int64_t)n * n;
  const int r = it.i + threadIdx.x;
  for (int j0 = 0; j0 < nrhs; j0 += 64) {
    const int nj = min(64, nrhs - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < b * nj; e += 256) {
      const int a = e % b, j = e / b;
      const int64_t o = k + a + (int64_t)(j0 + j) * n;
      sr[a][j] = vr[o];
      si[a][j] = vi[o];
    }
    __syncthreads();
    if (r < n) row_update(sr, si, fr, fi, vr, vi, n, k, b, r, j0, nj);
  }
}

template <typename T>
__device__ __forceinline__ void apply_dinv(const KP<T> &p, const FrontDev &f, T *vr, T *vi, int nrhs);

// z = D^-1 y over the fully-summed positions
template <typename T>
__global__ __launch_bounds__(256) void k_ffin(KP<T> p, int64_t first, int nrhs) {
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)f.n * p.mr;
  apply_dinv(p, f, vr, vi, nrhs);
}

template <typename T>
__global__ __launch_bounds__(256) void k_binit(KP<T> p, int64_t first, int nrhs) {
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, s = f.s, R = n - s;
  const int64_t mr = p.mr;
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)n * mr;
  const bool aux = f.kind == FK_AUX;
  const int64_t ld = aux ? p.n_mult : p.n_torn;
  const T *sr = p.num + (aux ? p.vl : p.vx);
  const T *si = sr + ld * mr;
  for (int e = threadIdx.x; e < R * nrhs; e += 256) {
    const int r = s + e % R, j = e / R;
    const int64_t row = f.vbase + p.vars[f.idx + r] + (int64_t)j * ld;
    vr[r + (int64_t)j * n] = sr[row];
    vi[r + (int64_t)j * n] = si[row];
  }
}

// Accumulates sum_{r in [r0, r1)} L(r, k + c) x(r, j) for c = tid % 64 and
// j = j0 + 4 (tid / 64) + q into (ar, ai), staging 64-row chunks in LDS.
template <typename T>
__device__ __forceinline__ void col_dot(T (&lr)[64][NB + 1], T (&li)[64][NB + 1], T (&xr)[64][17], T (&xi)[64][17],
                                        const T *fr, const T *fi, const T *vr, const T *vi, int n, int k, int b,
                                        int r0, int r1, int j0, int nrhs, T (&ar)[4], T (&ai)[4]) {
  const int tid = threadIdx.x, c = tid & 63, jg = tid >> 6;
  for (int rb = r0; rb < r1; rb += 64) {
    const int rows = min(64, r1 - rb);
    __syncthreads();
    for (int e = tid; e < 64 * NB; e += 256) {
      const int m = e % 64, cc = e / 64;
      T a = 0, bb = 0;
      if (m < rows && cc < b) {
        const int64_t o = (rb + m) + (int64_t)(k + cc) * n;
        a = fr[o];
        bb = fi[o];
      }
      lr[m][cc] = a;
      li[m][cc] = bb;
    }
    for (int e = tid; e < 64 * 16; e += 256) {
      const int m = e % 64, j = e / 64;
      T a = 0, bb = 0;
      if (m < rows && j0 + j < nrhs) {
        const int64_t o = (rb + m) + (int64_t)(j0 + j) * n;
        a = vr[o];
        bb = vi[o];
      }
      xr[m][j] = a;
      xi[m][j] = bb;
    }
    __syncthreads();
    for (int m = 0; m < rows; ++m) {
      const T a = lr[m][c], bb = li[m][c];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = jg * 4 + q;
        ar[q] += a * xr[m][j] - bb * xi[m][j];
        ai[q] += a * xi[m][j] + bb * xr[m][j];
      }
    }
  }
}

// partial[slot](c, j) = sum over rows [r0, r0 + 256) of L(r, k + c) x(r, j)
template <typename T>
__global__ __launch_bounds__(256) void k_bpart(KP<T> p, int64_t first, int nrhs) {
  __shared__ T lr[64][NB + 1], li[64][NB + 1];
  __shared__ T xr[64][17], xi[64][17];
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, k = it.k, b = min(NB, f.s - k), r0 = it.i;
  const int64_t mr = p.mr;
  const T *vr = p.num + f.voff;
  const T *vi = vr + (int64_t)n * mr;
  const T *fr = p.num + f.off;
  const T *fi = fr + (int64_t)n * n;
  T *pr = p.num + p.part + (int64_t)it.j * NB * mr * 2;
  T *pi = pr + (int64_t)NB * mr;
  const int c = threadIdx.x & 63, jg = threadIdx.x >> 6;
  for (int j0 = 0; j0 < nrhs; j0 += 16) {
    T ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
    col_dot(lr, li, xr, xi, fr, fi, vr, vi, n, k, b, r0, min(r0 + 256, n), j0, nrhs, ar, ai);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + jg * 4 + q;
      if (c < b && j < nrhs) {
        pr[c + (int64_t)j * NB] = ar[q];
        pi[c + (int64_t)j * NB] = ai[q];
      }
    }
  }
}

// v(k + c, j) -= sum_{r >= k+b} L(r, k + c) x(r, j) for the 8 columns
// c in [c0, c0 + 8) of pivot tile k: 32 lanes per column stride over the rows,
// the lane sums are reduced through LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_bcol(KP<T> p, int64_t first, int nrhs) {
  __shared__ T rr_[8][32][17], ri_[8][32][17];
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, k = it.k, b = min(NB, f.s - k);
  const int64_t mr = p.mr;
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)n * mr;
  const T *fr = p.num + f.off;
  const T *fi = fr + (int64_t)n * n;
  const int cl = threadIdx.x >> 5, lane = threadIdx.x & 31;
  const int c = it.i + cl;
  const bool live = c < b;
  const T *Lr = fr + (int64_t)(k + (live ? c : 0)) * n;
  const T *Li = fi + (int64_t)(k + (live ? c : 0)) * n;
  for (int j0 = 0; j0 < nrhs; j0 += 16) {
    const int nj = min(16, nrhs - j0);
    T ar[16], ai[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) ar[q] = ai[q] = 0;
    if (live) {
      for (int r = k + b + lane; r < n; r += 32) {
        const T lr = Lr[r], li = Li[r];
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (q < nj) {
            const int64_t o = r + (int64_t)(j0 + q) * n;
            const T xr = vr[o], xi = vi[o];
            ar[q] += lr * xr - li * xi;
            ai[q] += lr * xi + li * xr;
          }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      rr_[cl][lane][q] = ar[q];
      ri_[cl][lane][q] = ai[q];
    }
    __syncthreads();
    if (threadIdx.x < 8 * 16) {
      const int cc = threadIdx.x >> 4, q = threadIdx.x & 15;
      if (it.i + cc < b && q < nj) {
        T sr = 0, si = 0;
#pragma unroll 8
        for (int l = 0; l < 32; ++l) {
          sr += rr_[cc][l][q];
          si += ri_[cc][l][q];
        }
        const int64_t o = k + it.i + cc + (int64_t)(j0 + q) * n;
        vr[o] -= sr;
        vi[o] -= si;
      }
    }
  }
}

// x_k = P_k^T L_kk^-T z for columns [j0, j0 + nj) (z in zr/zi, ld 65)
template <typename T, int ZC>
__device__ __forceinline__ void tile_backward(const T (&zr)[NB][ZC], const T (&zi)[NB][ZC],
                                              const T (&yr)[NB][NB + 1], const T (&yi)[NB][NB + 1], T *vr, T *vi,
                                              int n, int k, int b, const int32_t *pm, int j0, int nj) {
  for (int e = threadIdx.x; e < b * nj; e += 256) {
    const int a = e % b, j = e / b;
    T wr = zr[a][j], wi = zi[a][j];
    for (int c = a + 1; c < b; ++c) {
      const T lr = yr[c][a], li = yi[c][a];
      wr += lr * zr[c][j] - li * zi[c][j];
      wi += lr * zi[c][j] + li * zr[c][j];
    }
    const int64_t o = k + pm[a] + (int64_t)(j0 + j) * n;
    vr[o] = wr;
    vi[o] = wi;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_bdiag(KP<T> p, int64_t first, int nrhs) {
  __shared__ T zr[NB][65], zi[NB][65];
  __shared__ T yr[NB][NB + 1], yi[NB][NB + 1];
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, k = it.k, b = min(NB, f.s - k);
  const int64_t mr = p.mr;
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)n * mr;
  const T *fr = p.num + f.off;
  const T *fi = fr + (int64_t)n * n;
  load_ytile(yr, yi, fr, fi, n, k, b);
  for (int j0 = 0; j0 < nrhs; j0 += 64) {
    const int nj = min(64, nrhs - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < b * nj; e += 256) {
      const int a = e % b, j = e / b;
      const int64_t o = k + a + (int64_t)(j0 + j) * n;
      T sr = vr[o], si = vi[o];
      const int64_t q = a + (int64_t)(j0 + j) * NB;
      const T *pr = p.num + p.part + (int64_t)it.i * NB * mr * 2 + q;
      const int64_t stride = (int64_t)NB * mr * 2;
      int sl = 0;
      for (; sl + 4 <= it.j; sl += 4) {
        T x0 = pr[(sl + 0) * stride], x1 = pr[(sl + 1) * stride], x2 = pr[(sl + 2) * stride],
          x3 = pr[(sl + 3) * stride];
        T y0 = pr[(sl + 0) * stride + NB * mr], y1 = pr[(sl + 1) * stride + NB * mr],
          y2 = pr[(sl + 2) * stride + NB * mr], y3 = pr[(sl + 3) * stride + NB * mr];
        sr -= (x0 + x1) + (x2 + x3);
        si -= (y0 + y1) + (y2 + y3);
      }
      for (; sl < it.j; ++sl) {
        sr -= pr[sl * stride];
        si -= pr[sl * stride + NB * mr];
      }
      zr[a][j] = sr;
      zi[a][j] = si;
    }
    __syncthreads();
    tile_backward(zr, zi, yr, yi, vr, vi, n, k, b, p.perm + f.soff + k, j0, nj);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_bfin(KP<T> p, int64_t first, int nrhs) {
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, s = f.s;
  const int64_t mr = p.mr;
  const T *vr = p.num + f.voff;
  const T *vi = vr + (int64_t)n * mr;
  const bool aux = f.kind == FK_AUX;
  const int64_t ld = aux ? p.n_mult : p.n_torn;
  T *dr = p.num + (aux ? p.vl : p.vx);
  T *di = dr + ld * mr;
  for (int e = threadIdx.x; e < s * nrhs; e += 256) {
    const int r = e % s, j = e / s;
    const int64_t row = f.vbase + p.vars[f.idx + r] + (int64_t)j * ld;
    dr[row] = vr[r + (int64_t)j * n];
    di[row] = vi[r + (int64_t)j * n];
  }
}

// z = D^-1 y over the fully-summed positions of one front (block-wide loop)
template <typename T>
__device__ __forceinline__ void apply_dinv(const KP<T> &p, const FrontDev &f, T *vr, T *vi, int nrhs) {
  const int n = f.n, s = f.s;
  for (int e = threadIdx.x; e < s * nrhs; e += 256) {
    const int a = e % s, j = e / s;
    const int64_t sa = f.soff + a;
    const int pd = p.pdel[sa];
    if (pd < 0) continue;
    const int64_t o = a + (int64_t)j * n;
    const cd d = p.dinv[sa];
    const double y0r = vr[o], y0i = vi[o];
    if (pd == 0) {
      vr[o] = (T)(d.re * y0r - d.im * y0i);
      vi[o] = (T)(d.re * y0i + d.im * y0r);
    } else {
      const cd d1 = p.dinv[sa + 1], od = p.doff[sa];
      const double y1r = vr[o + 1], y1i = vi[o + 1];
      vr[o] = (T)((d.re * y0r - d.im * y0i) + (od.re * y1r - od.im * y1i));
      vi[o] = (T)((d.re * y0i + d.im * y0r) + (od.re * y1i + od.im * y1r));
      vr[o + 1] = (T)((od.re * y0r - od.im * y0i) + (d1.re * y1r - d1.im * y1i));
      vi[o + 1] = (T)((od.re * y0i + od.im * y0r) + (d1.re * y1i + d1.im * y1r));
    }
  }
}

// Whole-front forward substitution in one workgroup (fronts up to FUSE_N):
// gather + children updates, then per pivot tile y_k = L_kk^-1 P_k v_k and
// v(rows below) -= L21 y_k, finally z = D^-1 y.
template <typename T>
__global__ __launch_bounds__(256) void k_ffront(KP<T> p, int64_t first, int nrhs) {
  __shared__ T sr[NB][65], si[NB][65];
  __shared__ T yr[NB][NB + 1], yi[NB][NB + 1];
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, s = f.s, tid = threadIdx.x;
  const int64_t mr = p.mr;
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)n * mr;
  const T *fr = p.num + f.off;
  const T *fi = fr + (int64_t)n * n;
  {
    const bool aux = f.kind == FK_AUX;
    const int64_t ld = aux ? p.n_mult : p.n_torn;
    const T *gr = p.num + (aux ? p.vd : p.vf);
    const T *gi = gr + ld * mr;
    for (int e = tid; e < n * nrhs; e += 256) {
      const int r = e % n, j = e / n;
      T xr = 0, xi = 0;
      if (r < s) {
        const int64_t row = f.vbase + p.vars[f.idx + r] + (int64_t)j * ld;
        xr = gr[row];
        xi = gi[row];
      }
      for (int ch = 0; ch < f.nchild; ++ch) {
        const int rr = p.rmap[p.crmap[f.child + ch] + r];
        if (rr < 0) continue;
        const FrontDev &cf = p.F[p.cfront[f.child + ch]];
        const int64_t o = cf.voff + cf.s + rr + (int64_t)j * cf.n;
        xr += p.num[o];
        xi += p.num[o + (int64_t)cf.n * mr];
      }
      vr[r + (int64_t)j * n] = xr;
      vi[r + (int64_t)j * n] = xi;
    }
  }
  for (int k = 0; k < s; k += NB) {
    const int b = min(NB, s - k);
    __syncthreads();
    load_ytile(yr, yi, fr, fi, n, k, b);
    for (int j0 = 0; j0 < nrhs; j0 += 64) {
      const int nj = min(64, nrhs - j0);
      tile_forward(sr, si, yr, yi, vr, vi, n, k, b, p.perm + f.soff + k, j0, nj);
      for (int r = k + b + tid; r < n; r += 256) row_update(sr, si, fr, fi, vr, vi, n, k, b, r, j0, nj);
      __syncthreads();
    }
  }
  __syncthreads();
  apply_dinv(p, f, vr, vi, nrhs);
}

// Whole-front backward substitution in one workgroup: x_R gathered from the
// global solution, then per pivot tile (descending) x_k = P_k^T L_kk^-T
// (z_k - L21^T x_below), finally the fully-summed part is scattered.
template <typename T>
__global__ __launch_bounds__(256) void k_bfront(KP<T> p, int64_t first, int nrhs) {
  __shared__ T lr[64][NB + 1], li[64][NB + 1];
  __shared__ T xr[64][17], xi[64][17];
  __shared__ T zr[NB][17], zi[NB][17];
  // the diagonal-tile inverse is staged in the same LDS as the L chunks
  T (&yr)[NB][NB + 1] = lr;
  T (&yi)[NB][NB + 1] = li;
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, s = f.s, R = n - s, tid = threadIdx.x;
  const int64_t mr = p.mr;
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)n * mr;
  const T *fr = p.num + f.off;
  const T *fi = fr + (int64_t)n * n;
  const bool aux = f.kind == FK_AUX;
  const int64_t ld = aux ? p.n_mult : p.n_torn;
  {
    const T *gr = p.num + (aux ? p.vl : p.vx);
    const T *gi = gr + ld * mr;
    for (int e = tid; e < R * nrhs; e += 256) {
      const int r = s + e % R, j = e / R;
      const int64_t row = f.vbase + p.vars[f.idx + r] + (int64_t)j * ld;
      vr[r + (int64_t)j * n] = gr[row];
      vi[r + (int64_t)j * n] = gi[row];
    }
  }
  const int c = tid & 63, jg = tid >> 6;
  const int T0 = (s + NB - 1) / NB;
  for (int t = T0 - 1; t >= 0; --t) {
    const int k = t * NB, b = min(NB, s - k);
    for (int j0 = 0; j0 < nrhs; j0 += 16) {
      T ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
      col_dot(lr, li, xr, xi, fr, fi, vr, vi, n, k, b, k + b, n, j0, nrhs, ar, ai);
      __syncthreads();
      load_ytile(yr, yi, fr, fi, n, k, b);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = jg * 4 + q;
        T zr_ = 0, zi_ = 0;
        if (c < b && j0 + j < nrhs) {
          const int64_t o = k + c + (int64_t)(j0 + j) * n;
          zr_ = vr[o] - ar[q];
          zi_ = vi[o] - ai[q];
        }
        zr[c][j] = zr_;
        zi[c][j] = zi_;
      }
      __syncthreads();
      tile_backward(zr, zi, yr, yi, vr, vi, n, k, b, p.perm + f.soff + k, j0, min(16, nrhs - j0));
    }
  }
  __syncthreads();
  T *dr = p.num + (aux ? p.vl : p.vx);
  T *di = dr + ld * mr;
  for (int e = tid; e < s * nrhs; e += 256) {
    const int r = e % s, j = e / s;
    const int64_t row = f.vbase + p.vars[f.idx + r] + (int64_t)j * ld;
    dr[row] = vr[r + (int64_t)j * n];
    di[row] = vi[r + (int64_t)j * n];
  }
}

// Substitutions through a front whose fully-summed block carries Z = L^-1
// (formed during the factorisation, P basis, lower triangle, unit diagonal).
// Forward:  y = Z (P v_s) into the W scratch; then v_s = y and v_R -= L21 y.
// Backward: t = z - L21^T x_R into the W scratch; x_s = P^T Z^T t.
// Workgroups own 64 rows (or 64 columns); 4 thread groups split the inner
// dimension and are reduced through LDS.  The right-hand side of the inner
// products is staged in LDS in chunks of 256.
template <typename T>
__device__ __forceinline__ void rows_dot(const KP<T> &p, const FrontDev &f, int r0, int kbeg, int kend, bool tri,
                                         bool perm_in, const T *inr, const T *ini, int64_t ldin, int j0, int nj,
                                         T (&ar)[8], T (&ai)[8], T (&sr)[256][9], T (&si)[256][9]) {
  // ar/ai(q) = sum_{c in [kbeg, kend)} A(r0 + m, c) in(c', j0 + q) for row m = tid % 64
  // A = Z (tri: c <= r, unit diagonal) or L (front entries); c' = P(c) if perm_in
  const int n = f.n, m = threadIdx.x & 63, cg = threadIdx.x >> 6, r = r0 + m;
  const T *fr = p.num + f.off;
  const T *fi = fr + (int64_t)n * n;
  const int32_t *pm = p.perm + f.soff;
#pragma unroll
  for (int q = 0; q < 8; ++q) ar[q] = ai[q] = 0;
  for (int c0 = kbeg; c0 < kend; c0 += 256) {
    __syncthreads();
    for (int e = threadIdx.x; e < 256 * 8; e += 256) {
      const int c = e % 256, q = e / 256;
      T br = 0, bi = 0;
      if (c0 + c < kend && q < nj) {
        const int cc = c0 + c;
        const int src = perm_in ? (cc / NB) * NB + pm[cc] : cc;
        const int64_t io = src + (int64_t)(j0 + q) * ldin;
        br = inr[io];
        bi = ini[io];
      }
      sr[c][q] = br;
      si[c][q] = bi;
    }
    __syncthreads();
    const int cend = min(256, kend - c0);
    if (r < n) {
      for (int c = cg; c < cend; c += 4) {
        const int cc = c0 + c;
        T xr = 0, xi = 0;
        if (!tri || cc < r) {
          const int64_t o = r + (int64_t)cc * n;
          xr = fr[o];
          xi = fi[o];
        } else if (cc == r) {
          xr = 1;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          ar[q] += xr * sr[c][q] - xi * si[c][q];
          ai[q] += xr * si[c][q] + xi * sr[c][q];
        }
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ void reduce4(T (&ar)[8], T (&ai)[8], T (&rr)[4][64][9], T (&ri)[4][64][9]) {
  const int m = threadIdx.x & 63, cg = threadIdx.x >> 6;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    rr[cg][m][q] = ar[q];
    ri[cg][m][q] = ai[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    ar[q] = rr[0][m][q] + rr[1][m][q] + rr[2][m][q] + rr[3][m][q];
    ai[q] = ri[0][m][q] + ri[1][m][q] + ri[2][m][q] + ri[3][m][q];
  }
}

// y(rows r0..r0+64 of the fully-summed part) = Z (P v_s)  -> W scratch
template <typename T>
__global__ __launch_bounds__(256) void k_zfwd(KP<T> p, int64_t first, int nrhs) {
  __shared__ T sr[256][9], si[256][9];
  __shared__ T rr[4][64][9], ri[4][64][9];
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, s = f.s, r0 = it.i, m = threadIdx.x & 63, cg = threadIdx.x >> 6;
  const int64_t mr = p.mr;
  const T *vr = p.num + f.voff;
  const T *vi = vr + (int64_t)n * mr;
  T *Wr = p.num + f.woff;
  T *Wi = Wr + (int64_t)n * f.wcols;
  for (int j0 = 0; j0 < nrhs; j0 += 8) {
    const int nj = min(8, nrhs - j0);
    T ar[8], ai[8];
    rows_dot(p, f, r0, 0, min(r0 + 64, s), true, true, vr, vi, n, j0, nj, ar, ai, sr, si);
    reduce4(ar, ai, rr, ri);
    if (cg == 0 && r0 + m < s)
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < nj) {
          Wr[r0 + m + (int64_t)(j0 + q) * n] = ar[q];
          Wi[r0 + m + (int64_t)(j0 + q) * n] = ai[q];
        }
  }
}

// rows r0..r0+64: v_s = y (rows < s); v_R -= L21 y (rows >= s)
template <typename T>
__global__ __launch_bounds__(256) void k_zfwd2(KP<T> p, int64_t first, int nrhs) {
  __shared__ T sr[256][9], si[256][9];
  __shared__ T rr[4][64][9], ri[4][64][9];
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, s = f.s, r0 = it.i, m = threadIdx.x & 63, cg = threadIdx.x >> 6, r = r0 + m;
  const int64_t mr = p.mr;
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)n * mr;
  const T *Wr = p.num + f.woff;
  const T *Wi = Wr + (int64_t)n * f.wcols;
  if (r0 < s) {
    for (int e = threadIdx.x; e < 64 * nrhs; e += 256) {
      const int mm = e % 64, j = e / 64;
      if (r0 + mm < s) {
        vr[r0 + mm + (int64_t)j * n] = Wr[r0 + mm + (int64_t)j * n];
        vi[r0 + mm + (int64_t)j * n] = Wi[r0 + mm + (int64_t)j * n];
      }
    }
  }
  if (r0 + 64 <= s || r0 >= n) return;   // no update rows in this tile (uniform)
  for (int j0 = 0; j0 < nrhs; j0 += 8) {
    const int nj = min(8, nrhs - j0);
    T ar[8], ai[8];
    rows_dot(p, f, r0, 0, s, false, false, Wr, Wi, n, j0, nj, ar, ai, sr, si);
    reduce4(ar, ai, rr, ri);
    if (cg == 0 && r >= s && r < n)
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < nj) {
          vr[r + (int64_t)(j0 + q) * n] -= ar[q];
          vi[r + (int64_t)(j0 + q) * n] -= ai[q];
        }
  }
}

// t(columns c0..c0+64 of the fully-summed part) = z - L21^T x_R -> W scratch
template <typename T>
__global__ __launch_bounds__(256) void k_zbwd1(KP<T> p, int64_t first, int nrhs) {
  __shared__ T lr[64][NB + 1], li[64][NB + 1];
  __shared__ T xr[64][17], xi[64][17];
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, s = f.s, c0 = it.i, b = min(64, s - c0);
  const int64_t mr = p.mr;
  const T *vr = p.num + f.voff;
  const T *vi = vr + (int64_t)n * mr;
  const T *fr = p.num + f.off;
  const T *fi = fr + (int64_t)n * n;
  T *Wr = p.num + f.woff;
  T *Wi = Wr + (int64_t)n * f.wcols;
  const int c = threadIdx.x & 63, jg = threadIdx.x >> 6;
  for (int j0 = 0; j0 < nrhs; j0 += 16) {
    T ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
    if (s < n) col_dot(lr, li, xr, xi, fr, fi, vr, vi, n, c0, b, s, n, j0, nrhs, ar, ai);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + jg * 4 + q;
      if (c < b && j < nrhs) {
        const int64_t o = c0 + c + (int64_t)j * n;
        Wr[o] = vr[o] - ar[q];
        Wi[o] = vi[o] - ai[q];
      }
    }
  }
}

// x_s(columns a0..a0+64, P basis) = Z^T t, written un-permuted into v
template <typename T>
__global__ __launch_bounds__(256) void k_zbwd2(KP<T> p, int64_t first, int nrhs) {
  __shared__ T lr[64][NB + 1], li[64][NB + 1];
  __shared__ T xr[64][17], xi[64][17];
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, s = f.s, a0 = it.i, b = min(64, s - a0);
  const int64_t mr = p.mr;
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)n * mr;
  const T *fr = p.num + f.off;
  const T *fi = fr + (int64_t)n * n;
  const T *Wr = p.num + f.woff;
  const T *Wi = Wr + (int64_t)n * f.wcols;
  const int32_t *pm = p.perm + f.soff;
  const int a = threadIdx.x & 63, jg = threadIdx.x >> 6;
  for (int j0 = 0; j0 < nrhs; j0 += 16) {
    T ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
    // rows below the diagonal tile: plain column dot with Z
    if (a0 + 64 < s) col_dot(lr, li, xr, xi, fr, fi, Wr, Wi, n, a0, b, a0 + 64, s, j0, nrhs, ar, ai);
    // diagonal tile: Z(c, a) for c >= a (unit diagonal)
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int mm = e % 64, j = e / 64;
      T x0 = 0, x1 = 0;
      if (mm < b && j0 + j < nrhs) {
        const int64_t o = a0 + mm + (int64_t)(j0 + j) * n;
        x0 = Wr[o];
        x1 = Wi[o];
      }
      xr[mm][j] = x0;
      xi[mm][j] = x1;
    }
    __syncthreads();
    if (a < b) {
      for (int c = a; c < b; ++c) {
        T zr = 1, zi = 0;
        if (c > a) {
          const int64_t o = (a0 + c) + (int64_t)(a0 + a) * n;
          zr = fr[o];
          zi = fi[o];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = jg * 4 + q;
          ar[q] += zr * xr[c][j] - zi * xi[c][j];
          ai[q] += zr * xi[c][j] + zi * xr[c][j];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = j0 + jg * 4 + q;
        if (j < nrhs) {
          const int64_t o = (a0 / NB) * NB + pm[a0 + a] + (int64_t)j * n;
          vr[o] = ar[q];
          vi[o] = ai[q];
        }
      }
    }
  }
}

// interface GEMV: mode 0: YG = X v_root ; mode 1: v_root = YG - X h.
// Workgroup = 64 rows x 4 column groups; the right-hand side is staged in LDS
// in chunks of 256 columns of X.
template <typename T>
__global__ __launch_bounds__(256) void k_gemv(KP<T> p, int mode, int nrhs) {
  __shared__ T redr[4][64][9], redi[4][64][9];
  __shared__ T inr_s[256][9], ini_s[256][9];
  const Item it = p.gemv[blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int g = f.s;
  const int64_t mr = p.mr;
  const int m = threadIdx.x & 63, cg = threadIdx.x >> 6, r = it.i + m;
  const T *Xr = p.num + f.xoff;
  const T *Xi = Xr + (int64_t)g * g;
  const T *inr, *ini;
  T *outr, *outi;
  const T *addr = nullptr, *addi = nullptr;
  T *yg = p.num + f.goff;              // YG: re [g x mr], im after
  T *h = yg + 2 * (int64_t)g * mr;     // h
  T *v = p.num + f.voff;               // root vector (ld g)
  if (mode == 0) {
    inr = v; ini = v + (int64_t)g * mr;
    outr = yg; outi = yg + (int64_t)g * mr;
  } else {
    inr = h; ini = h + (int64_t)g * mr;
    addr = yg; addi = yg + (int64_t)g * mr;
    outr = v; outi = v + (int64_t)g * mr;
  }
  for (int j0 = 0; j0 < nrhs; j0 += 8) {
    const int nj = min(8, nrhs - j0);
    T ar[8], ai[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) ar[q] = ai[q] = 0;
    for (int c0 = 0; c0 < g; c0 += 256) {
      __syncthreads();
      for (int e = threadIdx.x; e < 256 * 8; e += 256) {
        const int c = e % 256, q = e / 256;
        T br = 0, bi = 0;
        if (c0 + c < g && q < nj) {
          const int64_t io = c0 + c + (int64_t)(j0 + q) * g;
          br = inr[io];
          bi = ini[io];
        }
        inr_s[c][q] = br;
        ini_s[c][q] = bi;
      }
      __syncthreads();
      if (r < g) {
        const int cend = min(256, g - c0);
        for (int c = cg; c < cend; c += 4) {
          const int64_t o = r + (int64_t)(c0 + c) * g;
          const T xr = Xr[o], xi = Xi[o];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            ar[q] += xr * inr_s[c][q] - xi * ini_s[c][q];
            ai[q] += xr * ini_s[c][q] + xi * inr_s[c][q];
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      redr[cg][m][q] = ar[q];
      redi[cg][m][q] = ai[q];
    }
    __syncthreads();
    if (cg == 0 && r < g) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (q >= nj) break;
        T sr = redr[0][m][q] + redr[1][m][q] + redr[2][m][q] + redr[3][m][q];
        T si = redi[0][m][q] + redi[1][m][q] + redi[2][m][q] + redi[3][m][q];
        const int64_t o = r + (int64_t)(j0 + q) * g;
        if (mode == 0) {
          outr[o] = sr;
          outi[o] = si;
        } else {
          outr[o] = addr[o] - sr;
          outi[o] = addi[o] - si;
        }
      }
    }
  }
}

// d(p) = sum_t s_t YG_t - c(p)
template <typename T>
__global__ __launch_bounds__(256) void k_mgather(KP<T> p, int nrhs, int with_c) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= p.n_mult * nrhs) return;
  const int64_t m = e % p.n_mult, j = e / p.n_mult;
  const MultRef R = p.mrefs[m];
  const int64_t mr = p.mr;
  T sr = 0, si = 0;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const T *y = p.num + R.o[t] + j * R.g[t];
    const T yr = y[0], yi = y[(int64_t)R.g[t] * mr];
    sr += R.sg[t] > 0 ? yr : -yr;
    si += R.sg[t] > 0 ? yi : -yi;
  }
  T *dr = p.num + p.vd;
  T *di = dr + p.n_mult * mr;
  if (with_c) {
    const T *cr = p.num + p.vc;
    sr -= cr[m + j * p.n_mult];
    si -= cr[m + j * p.n_mult + p.n_mult * mr];
  }
  dr[m + j * p.n_mult] = sr;
  di[m + j * p.n_mult] = si;
}

// h(gamma) = sum over multipliers on that dof of sign * lambda
template <typename T>
__global__ __launch_bounds__(256) void k_hgather(KP<T> p, int64_t ngam, int nrhs) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= ngam * nrhs) return;
  const int64_t q = e % ngam, j = e / ngam;
  const GamRef G = p.grefs[q];
  const int64_t mr = p.mr;
  const T *lr = p.num + p.vl;
  const T *li = lr + p.n_mult * mr;
  T sr = 0, si = 0;
  for (int t = 0; t < G.cnt; ++t) {
    const int64_t m = p.hmult[G.beg + t] + j * p.n_mult;
    const int sg = p.hsign[G.beg + t];
    sr += sg > 0 ? lr[m] : -lr[m];
    si += sg > 0 ? li[m] : -li[m];
  }
  T *h = p.num + G.o + j * G.g;
  h[0] = sr;
  h[(int64_t)G.g * mr] = si;
}

// ---------------------------------------------------------------------------
// conversions and FP64 refinement
template <typename T>
__global__ void k_f2t(KP<T> p, const cd *f, int64_t ldf, int nrhs) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= p.n_torn * nrhs) return;
  const int64_t r = e % p.n_torn, j = e / p.n_torn;
  const cd v = f[r + j * ldf];
  T *d = p.num + p.vf;
  d[r + j * p.n_torn] = (T)v.re;
  d[r + j * p.n_torn + p.n_torn * p.mr] = (T)v.im;
}

template <typename T>
__global__ void k_t2u(KP<T> p, cd *u, int64_t ldu, int nrhs, int which) {
  // which 0: VX -> u (n_torn rows); 1: VL -> u (n_mult rows)
  const int64_t rows = which ? p.n_mult : p.n_torn;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * nrhs) return;
  const int64_t r = e % rows, j = e / rows;
  const T *s = p.num + (which ? p.vl : p.vx);
  u[r + j * ldu] = cd{(double)s[r + j * rows], (double)s[r + j * rows + rows * p.mr]};
}

template <typename T>
__global__ void k_xinv_out(KP<T> p, int f_id, cd *out) {
  const FrontDev f = p.F[f_id];
  const int64_t g = f.s;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= g * g) return;
  const T *X = p.num + f.xoff;
  out[e] = cd{(double)X[e], (double)X[e + g * g]};
}

// FP64 refinement state: U (torn x mr planar doubles), L (mult x mr planar)
template <typename T>
__global__ void k_r_init(KP<T> p, int nrhs) {
  const int64_t mr = p.mr;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nt = p.n_torn * nrhs, nm = p.n_mult * nrhs;
  double *U = p.r64;
  double *L = U + 2 * p.n_torn * mr;
  if (e < nt) {
    const int64_t r = e % p.n_torn, j = e / p.n_torn;
    const T *x = p.num + p.vx;
    U[r + j * p.n_torn] = x[r + j * p.n_torn];
    U[r + j * p.n_torn + p.n_torn * mr] = x[r + j * p.n_torn + p.n_torn * mr];
  } else if (e < nt + nm) {
    const int64_t q = e - nt, m = q % p.n_mult, j = q / p.n_mult;
    const T *l = p.num + p.vl;
    L[m + j * p.n_mult] = l[m + j * p.n_mult];
    L[m + j * p.n_mult + p.n_mult * mr] = l[m + j * p.n_mult + p.n_mult * mr];
  }
}

template <typename T>
__global__ void k_r_update(KP<T> p, int nrhs) {
  const int64_t mr = p.mr;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nt = p.n_torn * nrhs, nm = p.n_mult * nrhs;
  double *U = p.r64;
  double *L = U + 2 * p.n_torn * mr;
  if (e < nt) {
    const int64_t r = e % p.n_torn, j = e / p.n_torn;
    const T *x = p.num + p.vx;
    U[r + j * p.n_torn] += (double)x[r + j * p.n_torn];
    U[r + j * p.n_torn + p.n_torn * mr] += (double)x[r + j * p.n_torn + p.n_torn * mr];
  } else if (e < nt + nm) {
    const int64_t q = e - nt, m = q % p.n_mult, j = q / p.n_mult;
    const T *l = p.num + p.vl;
    L[m + j * p.n_mult] += (double)l[m + j * p.n_mult];
    L[m + j * p.n_mult + p.n_mult * mr] += (double)l[m + j * p.n_mult + p.n_mult * mr];
  }
}

// r_u = f - K u - B^T lam ; r_l = -B u ; writes the FP32 correction rhs (vf, vc)
// and per-block sums of |r|^2 (or |f|^2 when fnorm) per column.  Columns are
// processed 8 at a time so the operator is streamed once per 8 columns.
template <typename T>
__global__ __launch_bounds__(256) void k_r_resid(KP<T> p, const cd *f, int64_t ldf, int nrhs, int64_t part_off,
                                                 int fnorm) {
  __shared__ double red[8][256];
  const int64_t mr = p.mr;
  const double *U = p.r64;
  const double *L = U + 2 * p.n_torn * mr;
  double *part = p.r64 + part_off;
  const int64_t nrow = p.n_torn + p.n_mult;
  const int64_t nt = p.n_torn, nm = p.n_mult;
  for (int j0 = 0; j0 < nrhs; j0 += 8) {
    const int nj = min(8, nrhs - j0);
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nrow; e += (int64_t)gridDim.x * 256) {
      double rr[8], ri[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) rr[q] = ri[q] = 0;
      if (e < nt) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (q < nj) {
            const cd fv = f[e + (j0 + q) * ldf];
            rr[q] = fv.re;
            ri[q] = fv.im;
          }
        if (!fnorm) {
          for (int64_t z = p.csrp[e]; z < p.csrp[e + 1]; ++z) {
            const cd a = p.vals[z];
            const int64_t c = p.csrc[z];
#pragma unroll
            for (int q = 0; q < 8; ++q)
              if (q < nj) {
                const double ur = U[c + (j0 + q) * nt], ui = U[c + (j0 + q) * nt + nt * mr];
                rr[q] -= a.re * ur - a.im * ui;
                ri[q] -= a.re * ui + a.im * ur;
              }
          }
          const int gidx = p.rowgam[e];
          if (gidx >= 0) {
            const GamRef G = p.grefs[gidx];
            for (int t = 0; t < G.cnt; ++t) {
              const int64_t m = p.hmult[G.beg + t];
              const double sg = p.hsign[G.beg + t];
#pragma unroll
              for (int q = 0; q < 8; ++q)
                if (q < nj) {
                  rr[q] -= sg * L[m + (j0 + q) * nm];
                  ri[q] -= sg * L[m + (j0 + q) * nm + nm * mr];
                }
            }
          }
          T *vf = p.num + p.vf;
#pragma unroll
          for (int q = 0; q < 8; ++q)
            if (q < nj) {
              vf[e + (j0 + q) * nt] = (T)rr[q];
              vf[e + (j0 + q) * nt + nt * mr] = (T)ri[q];
            }
        }
      } else if (!fnorm) {
        const int64_t m = e - nt;
        const MultRef R = p.mrefs[m];
        T *vc = p.num + p.vc;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (q < nj) {
            for (int t = 0; t < 2; ++t) {
              const double sg = R.sg[t];
              rr[q] -= sg * U[R.row[t] + (j0 + q) * nt];
              ri[q] -= sg * U[R.row[t] + (j0 + q) * nt + nt * mr];
            }
            vc[m + (j0 + q) * nm] = (T)rr[q];
            vc[m + (j0 + q) * nm + nm * mr] = (T)ri[q];
          }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] += rr[q] * rr[q] + ri[q] * ri[q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (threadIdx.x < st)
#pragma unroll
        for (int q = 0; q < 8; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x < nj) part[blockIdx.x + (int64_t)(j0 + threadIdx.x) * gridDim.x] = red[threadIdx.x][0];
    __syncthreads();
  }
}

__global__ void k_r_reduce(const double *part, int nblk, int nrhs, double *out) {
  const int j = blockIdx.x;
  if (j >= nrhs) return;
  __shared__ double red[256];
  double a = 0;
  for (int b = threadIdx.x; b < nblk; b += 256) a += part[b + (int64_t)j * nblk];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

template <typename T>
__global__ void k_r_out(KP<T> p, cd *u, int64_t ldu, cd *lam, int64_t ldl, int nrhs) {
  const int64_t mr = p.mr;
  const double *U = p.r64;
  const double *L = U + 2 * p.n_torn * mr;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nt = p.n_torn * nrhs, nm = p.n_mult * nrhs;
  if (e < nt) {
    const int64_t r = e % p.n_torn, j = e / p.n_torn;
    u[r + j * ldu] = cd{U[r + j * p.n_torn], U[r + j * p.n_torn + p.n_torn * mr]};
  } else if (lam && e < nt + nm) {
    const int64_t q = e - nt, m = q % p.n_mult, j = q / p.n_mult;
    lam[m + j * ldl] = cd{L[m + j * p.n_mult], L[m + j * p.n_mult + p.n_mult * mr]};
  }
}

// ---------------------------------------------------------------------------
// host side
template <typename T>
static KP<T> make_kp(const Plan &P, uint8_t *ws, const void *vals) {
  KP<T> k;
  const uint8_t *m = ws + P.b_meta;
  k.F = (const FrontDev *)(m + P.m_fronts);
  k.items = (const Item *)(m + P.m_items);
  k.vars = (const int32_t *)(m + P.m_vars);
  k.cfront = (const int32_t *)(m + P.m_cfront);
  k.crmap = (const int64_t *)(m + P.m_crmap);
  k.rmap = (const int32_t *)(m + P.m_rmap);
  k.spairs = (const SPair *)(m + P.m_spairs);
  k.aux = (const AuxItem *)(m + P.m_aux);
  k.gpos = (const int32_t *)(m + P.m_gpos);
  k.gsign = (const int32_t *)(m + P.m_gsign);
  k.mrefs = (const MultRef *)(m + P.m_mrefs);
  k.grefs = (const GamRef *)(m + P.m_grefs);
  k.hmult = (const int32_t *)(m + P.m_hmult);
  k.hsign = (const int32_t *)(m + P.m_hsign);
  k.rowgam = (const int32_t *)(m + P.m_rowgam);
  k.csrp = (const int64_t *)(m + P.m_csrp);
  k.csrc = (const int32_t *)(m + P.m_csrc);
  k.gemv = (const Item *)(m + P.m_gemv);
  k.num = (T *)(ws + P.b_num);
  uint8_t *sd = ws + P.b_side;
  k.dinv = (cd *)sd;
  k.doff = (cd *)(sd + P.side_n * 16);
  k.pdel = (int32_t *)(sd + P.side_n * 32);
  k.perm = (int32_t *)(sd + P.side_n * 36);
  k.vals = (const cd *)vals;
  k.status = (int *)(ws + P.b_status);
  k.r64 = (double *)(ws + P.b_r64);
  k.vf = P.vf_off;
  k.vx = P.vx_off;
  k.vd = P.vd_off;
  k.vl = P.vl_off;
  k.vc = P.vc_off;
  k.part = P.part_off;
  k.n_torn = P.n_torn;
  k.n_mult = P.n_mult;
  k.mr = P.max_rhs;
  return k;
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename T>
static hipError_t run_seq(const Plan &P, const KP<T> &k, const std::vector<Launch> &seq, int nrhs, hipStream_t st,
                          KTimer *tm) {
  for (const Launch &L : seq) {
    dim3 g(L.count), b(256);
    const bool timed = tm && tm->kind == L.kind && tm->used + 2 <= tm->cap;
    hipEvent_t *ev = timed ? (hipEvent_t *)tm->ev : nullptr;
    if (timed) {
      (void)hipEventRecord(ev[tm->used], st);
      tm->launches++;
      tm->flops += L.flops;
    }
    switch (L.kind) {
      case L_ASM: hipLaunchKernelGGL(k_asm<T>, g, b, 0, st, k, L.first); break;
      case L_SCAT: hipLaunchKernelGGL(k_scat<T>, g, b, 0, st, k, L.first); break;
      case L_AUXG: hipLaunchKernelGGL(k_auxg<T>, g, b, 0, st, k, L.first); break;
      case L_PANEL: hipLaunchKernelGGL(k_panel<T>, g, b, 0, st, k, L.first); break;
      case L_TRSM: hipLaunchKernelGGL(k_trsm<T>, g, b, 0, st, k, L.first); break;
      case L_SYRK: hipLaunchKernelGGL(k_syrk<T>, g, b, 0, st, k, L.first); break;
      case L_ZREC1: hipLaunchKernelGGL(k_zrec1<T>, g, b, 0, st, k, L.first); break;
      case L_ZREC2: hipLaunchKernelGGL(k_zrec2<T>, g, b, 0, st, k, L.first); break;
      case L_INVSYRK: hipLaunchKernelGGL(k_invsyrk<T>, g, b, 0, st, k, L.first); break;
      case S_FINIT: hipLaunchKernelGGL(k_finit<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_FDIAG: hipLaunchKernelGGL(k_fdiag<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_FUPD: hipLaunchKernelGGL(k_fupd<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_FFIN: hipLaunchKernelGGL(k_ffin<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_BINIT: hipLaunchKernelGGL(k_binit<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_BPART: hipLaunchKernelGGL(k_bpart<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_BDIAG: hipLaunchKernelGGL(k_bdiag<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_BFIN: hipLaunchKernelGGL(k_bfin<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_FFRONT: hipLaunchKernelGGL(k_ffront<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_BCOL: hipLaunchKernelGGL(k_bcol<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_ZFWD: hipLaunchKernelGGL(k_zfwd<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_ZFWD2: hipLaunchKernelGGL(k_zfwd2<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_ZBWD1: hipLaunchKernelGGL(k_zbwd1<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_ZBWD2: hipLaunchKernelGGL(k_zbwd2<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_BFRONT: hipLaunchKernelGGL(k_bfront<T>, g, b, 0, st, k, L.first, nrhs); break;
      default: return hipErrorInvalidValue;
    }
    if (timed) {
      (void)hipEventRecord(ev[tm->used + 1], st);
      tm->used += 2;
    }
  }
  return hipGetLastError();
}

// clears the status words (a kernel, so that graph capture records no memset)
__global__ void k_zero_status(int *status) {
  if (threadIdx.x < 2) status[threadIdx.x] = 0;
}

template <typename T>
static hipError_t factor_t(const Plan &P, uint8_t *ws, const void *vals, hipStream_t st, KTimer *tm) {
  KP<T> k = make_kp<T>(P, ws, vals);
  hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(64), 0, st, k.status);
  return run_seq<T>(P, k, P.factor_seq, 0, st, tm);
}

template <typename T>
static hipError_t solve_core_t(const Plan &P, uint8_t *ws, int nrhs, bool with_c, hipStream_t st, KTimer *tm) {
  KP<T> k = make_kp<T>(P, ws, nullptr);
  hipError_t e = run_seq<T>(P, k, P.solve_dom_fwd, nrhs, st, tm);
  if (e != hipSuccess) return e;
  if (!P.gemv_items.empty())
    hipLaunchKernelGGL(k_gemv<T>, dim3(P.gemv_items.size()), dim3(256), 0, st, k, 0, nrhs);
  if (P.n_mult > 0)
    hipLaunchKernelGGL(k_mgather<T>, dim3(nblk(P.n_mult * nrhs)), dim3(256), 0, st, k, nrhs, with_c ? 1 : 0);
  e = run_seq<T>(P, k, P.solve_aux, nrhs, st, tm);
  if (e != hipSuccess) return e;
  if (!P.grefs.empty())
    hipLaunchKernelGGL(k_hgather<T>, dim3(nblk((int64_t)P.grefs.size() * nrhs)), dim3(256), 0, st, k,
                       (int64_t)P.grefs.size(), nrhs);
  if (!P.gemv_items.empty())
    hipLaunchKernelGGL(k_gemv<T>, dim3(P.gemv_items.size()), dim3(256), 0, st, k, 1, nrhs);
  e = run_seq<T>(P, k, P.solve_dom_bwd, nrhs, st, tm);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t factor(const Plan &P, uint8_t *ws, const void *vals, hipStream_t st, KTimer *tm) {
  return P.precision == 0 ? factor_t<double>(P, ws, vals, st, tm) : factor_t<float>(P, ws, vals, st, tm);
}

hipError_t rhs_in(const Plan &P, uint8_t *ws, const void *f, int64_t ldf, int nrhs, hipStream_t st) {
  if (P.precision == 0)
    hipLaunchKernelGGL(k_f2t<double>, dim3(nblk(P.n_torn * nrhs)), dim3(256), 0, st, make_kp<double>(P, ws, nullptr),
                       (const cd *)f, ldf, nrhs);
  else
    hipLaunchKernelGGL(k_f2t<float>, dim3(nblk(P.n_torn * nrhs)), dim3(256), 0, st, make_kp<float>(P, ws, nullptr),
                       (const cd *)f, ldf, nrhs);
  return hipGetLastError();
}

hipError_t solve_core(const Plan &P, uint8_t *ws, int nrhs, bool with_c, hipStream_t st, KTimer *tm) {
  return P.precision == 0 ? solve_core_t<double>(P, ws, nrhs, with_c, st, tm)
                          : solve_core_t<float>(P, ws, nrhs, with_c, st, tm);
}

hipError_t sol_out(const Plan &P, uint8_t *ws, void *u, int64_t ldu, void *lam, int64_t ldl, int nrhs,
                   hipStream_t st) {
  if (P.precision == 0) {
    KP<double> k = make_kp<double>(P, ws, nullptr);
    hipLaunchKernelGGL(k_t2u<double>, dim3(nblk(P.n_torn * nrhs)), dim3(256), 0, st, k, (cd *)u, ldu, nrhs, 0);
    if (lam && P.n_mult)
      hipLaunchKernelGGL(k_t2u<double>, dim3(nblk(P.n_mult * nrhs)), dim3(256), 0, st, k, (cd *)lam, ldl, nrhs, 1);
  } else {
    KP<float> k = make_kp<float>(P, ws, nullptr);
    hipLaunchKernelGGL(k_t2u<float>, dim3(nblk(P.n_torn * nrhs)), dim3(256), 0, st, k, (cd *)u, ldu, nrhs, 0);
    if (lam && P.n_mult)
      hipLaunchKernelGGL(k_t2u<float>, dim3(nblk(P.n_mult * nrhs)), dim3(256), 0, st, k, (cd *)lam, ldl, nrhs, 1);
  }
  return hipGetLastError();
}

hipError_t interface_inverse_out(const Plan &P, uint8_t *ws, int front, void *out, hipStream_t st) {
  const int64_t g = P.fronts[front].s;
  if (P.precision == 0)
    hipLaunchKernelGGL(k_xinv_out<double>, dim3(nblk(g * g)), dim3(256), 0, st, make_kp<double>(P, ws, nullptr),
                       front, (cd *)out);
  else
    hipLaunchKernelGGL(k_xinv_out<float>, dim3(nblk(g * g)), dim3(256), 0, st, make_kp<float>(P, ws, nullptr),
                       front, (cd *)out);
  return hipGetLastError();
}

// refinement helpers (FP32 factor precision only)
hipError_t refine_init(const Plan &P, uint8_t *ws, int nrhs, hipStream_t st) {
  KP<float> k = make_kp<float>(P, ws, ws + P.b_vals);
  hipLaunchKernelGGL(k_r_init<float>, dim3(nblk((P.n_torn + P.n_mult) * nrhs)), dim3(256), 0, st, k, nrhs);
  return hipGetLastError();
}
hipError_t refine_update(const Plan &P, uint8_t *ws, int nrhs, hipStream_t st) {
  KP<float> k = make_kp<float>(P, ws, ws + P.b_vals);
  hipLaunchKernelGGL(k_r_update<float>, dim3(nblk((P.n_torn + P.n_mult) * nrhs)), dim3(256), 0, st, k, nrhs);
  return hipGetLastError();
}
hipError_t refine_resid(const Plan &P, uint8_t *ws, const void *f, int64_t ldf, int nrhs, bool fnorm,
                        hipStream_t st) {
  KP<float> k = make_kp<float>(P, ws, ws + P.b_vals);
  const int nb = (int)P.r_nblk;
  hipLaunchKernelGGL(k_r_resid<float>, dim3(nb), dim3(256), 0, st, k, (const cd *)f, ldf, nrhs, P.r_part,
                     fnorm ? 1 : 0);
  double *r64 = (double *)(ws + P.b_r64);
  hipLaunchKernelGGL(k_r_reduce, dim3(nrhs), dim3(256), 0, st, r64 + P.r_part, nb, nrhs,
                     r64 + (fnorm ? P.r_fnorm : P.r_norm));
  return hipGetLastError();
}
hipError_t refine_out(const Plan &P, uint8_t *ws, void *u, int64_t ldu, void *lam, int64_t ldl, int nrhs,
                      hipStream_t st) {
  KP<float> k = make_kp<float>(P, ws, ws + P.b_vals);
  hipLaunchKernelGGL(k_r_out<float>, dim3(nblk((P.n_torn + P.n_mult) * nrhs)), dim3(256), 0, st, k, (cd *)u, ldu,
                     (cd *)lam, ldl, nrhs);
  return hipGetLastError();
}

}  // namespace dd
