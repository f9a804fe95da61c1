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
// assembly
template <typename T>
__global__ __launch_bounds__(256) void k_asm(KP<T> p, int64_t first) {
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n;
  T *re = p.num + f.off;
  T *im = re + (int64_t)n * n;
  const int cend = min(it.k + 64, n);
  for (int c = it.k; c < cend; ++c) {
    for (int r = c + threadIdx.x; r < n; r += 256) {
      T vr = 0, vi = 0;
      for (int ch = 0; ch < f.nchild; ++ch) {
        const int32_t *rm = p.rmap + p.crmap[f.child + ch];
        const int rc = rm[c];
        if (rc < 0) continue;
        const int rr = rm[r];
        if (rr < 0) continue;
        const FrontDev &cf = p.F[p.cfront[f.child + ch]];
        const int64_t o = cf.off + (cf.s + rr) + (int64_t)(cf.s + rc) * cf.n;
        vr += p.num[o];
        vi += p.num[o + (int64_t)cf.n * cf.n];
      }
      re[r + (int64_t)c * n] = vr;
      im[r + (int64_t)c * n] = vi;
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

// W' = P L_stored(rows r0.., tile k) L_kk^-1
template <typename T>
__global__ __launch_bounds__(256) void k_invprep(KP<T> p, int64_t first) {
  __shared__ GemmSmem<T> sm;
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int k = it.k, r0 = it.i, n = f.n;
  T *fr = p.num + f.off;
  T *fi = fr + (int64_t)n * n;
  const int32_t *pm = p.perm + f.soff;
  auto fa = [&](int m, int kk, T &re, T &im) {
    const int r = r0 + m;
    if (r < n) {
      const int rs = (r / NB) * NB + pm[r];
      const int64_t o = rs + (int64_t)(k + kk) * n;
      re = fr[o];
      im = fi[o];
    }
  };
  auto fb = [&](int c, int kk, T &re, T &im) {   // Y(kk, c), Y = L_kk^-1
    zval(fr, fi, n, k + kk, k + c, re, im);
  };
  typename V4<T>::t cr[2][2], ci[2][2];
  gemm_tile<T, false, true>(sm, 0, NB, fa, fb, cr, ci);
  T *Wr = p.num + f.woff;
  T *Wi = Wr + (int64_t)n * f.wcols;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = out_row(x), c = out_col<T>(y, i);
        if (r0 + m < n) {
          Wr[(r0 + m) + (int64_t)c * n] = cr[x][y][i];
          Wi[(r0 + m) + (int64_t)c * n] = ci[x][y][i];
        }
      }
}

// Z(r0.., tile k) = -Z22 W'
template <typename T>
__global__ __launch_bounds__(256) void k_invtrmm(KP<T> p, int64_t first) {
  __shared__ GemmSmem<T> sm;
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int k = it.k, r0 = it.i, n = f.n;
  T *fr = p.num + f.off;
  T *fi = fr + (int64_t)n * n;
  const T *Wr = p.num + f.woff;
  const T *Wi = Wr + (int64_t)n * f.wcols;
  auto fa = [&](int m, int kk, T &re, T &im) {
    const int r = r0 + m;
    if (r < n) zval(fr, fi, n, r, kk, re, im);
  };
  auto fb = [&](int c, int kk, T &re, T &im) {
    const int64_t o = kk + (int64_t)c * n;
    re = Wr[o];
    im = Wi[o];
  };
  typename V4<T>::t cr[2][2], ci[2][2];
  gemm_tile<T, false, true>(sm, k + NB, min(r0 + GT, n), fa, fb, cr, ci);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = out_row(x), c = out_col<T>(y, i);
        if (r0 + m < n) {
          const int64_t o = (r0 + m) + (int64_t)(k + c) * n;
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

// y_k = L_kk^-1 P_k v_k
template <typename T>
__global__ __launch_bounds__(256) void k_fdiag(KP<T> p, int64_t first, int nrhs) {
  __shared__ T sr[NB][65], si[NB][65];
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, k = it.k, b = min(NB, f.s - k);
  const int64_t mr = p.mr;
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)n * mr;
  const T *fr = p.num + f.off;
  const T *fi = fr + (int64_t)n * n;
  const int32_t *pm = p.perm + f.soff + k;
  for (int j0 = 0; j0 < nrhs; j0 += 64) {
    const int nj = min(64, nrhs - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < b * nj; e += 256) {
      const int a = e % b, j = e / b;
      const int64_t o = k + pm[a] + (int64_t)(j0 + j) * n;
      sr[a][j] = vr[o];
      si[a][j] = vi[o];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < b * nj; e += 256) {
      const int a = e % b, j = e / b;
      T yr = sr[a][j], yi = si[a][j];
      for (int c = 0; c < a; ++c) {
        const int64_t o = (k + a) + (int64_t)(k + c) * n;
        const T lr = fr[o], li = fi[o];
        yr += lr * sr[c][j] - li * si[c][j];
        yi += lr * si[c][j] + li * sr[c][j];
      }
      const int64_t o = k + a + (int64_t)(j0 + j) * n;
      vr[o] = yr;
      vi[o] = yi;
    }
  }
}

// v(rows r0..r0+255, r >= k+b) -= L21(:, tile k) y_k
template <typename T>
__global__ __launch_bounds__(256) void k_fupd(KP<T> p, int64_t first, int nrhs) {
  __shared__ T yr[NB][65], yi[NB][65];
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
      yr[a][j] = vr[o];
      yi[a][j] = vi[o];
    }
    __syncthreads();
    if (r < n) {
      for (int jj = 0; jj < nj; jj += 8) {
        T ar[8], ai[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) ar[q] = ai[q] = 0;
        for (int c = 0; c < b; ++c) {
          const int64_t o = r + (int64_t)(k + c) * n;
          const T lr = fr[o], li = fi[o];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            ar[q] += lr * yr[c][jj + q] - li * yi[c][jj + q];
            ai[q] += lr * yi[c][jj + q] + li * yr[c][jj + q];
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
  }
}

// z = D^-1 y over the fully-summed positions
template <typename T>
__global__ __launch_bounds__(256) void k_ffin(KP<T> p, int64_t first, int nrhs) {
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, s = f.s;
  const int64_t mr = p.mr;
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)n * mr;
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

// partial[slot](c, j) = sum_{r in chunk} L(r, k + c) x(r, j)
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
  const int rows = min(64, n - r0);
  for (int e = threadIdx.x; e < 64 * NB; e += 256) {
    const int m = e % 64, c = e / 64;
    T a = 0, bb = 0;
    if (m < rows && c < b) {
      const int64_t o = (r0 + m) + (int64_t)(k + c) * n;
      a = fr[o];
      bb = fi[o];
    }
    lr[m][c] = a;
    li[m][c] = bb;
  }
  const int c = threadIdx.x & 63, jg = threadIdx.x >> 6;
  for (int j0 = 0; j0 < nrhs; j0 += 16) {
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int m = e % 64, j = e / 64;
      T a = 0, bb = 0;
      if (m < rows && j0 + j < nrhs) {
        const int64_t o = (r0 + m) + (int64_t)(j0 + j) * n;
        a = vr[o];
        bb = vi[o];
      }
      xr[m][j] = a;
      xi[m][j] = bb;
    }
    __syncthreads();
    T ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
    for (int m = 0; m < rows; ++m) {
      const T a = lr[m][c], bb = li[m][c];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = jg * 4 + q;
        ar[q] += a * xr[m][j] - bb * xi[m][j];
        ai[q] += a * xi[m][j] + bb * xr[m][j];
      }
    }
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

// x_k = P_k^T L_kk^-T (z_k - sum partials)
template <typename T>
__global__ __launch_bounds__(256) void k_bdiag(KP<T> p, int64_t first, int nrhs) {
  __shared__ T zr[NB][65], zi[NB][65];
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, k = it.k, b = min(NB, f.s - k);
  const int64_t mr = p.mr;
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)n * mr;
  const T *fr = p.num + f.off;
  const T *fi = fr + (int64_t)n * n;
  const int32_t *pm = p.perm + f.soff + k;
  for (int j0 = 0; j0 < nrhs; j0 += 64) {
    const int nj = min(64, nrhs - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < b * nj; e += 256) {
      const int a = e % b, j = e / b;
      const int64_t o = k + a + (int64_t)(j0 + j) * n;
      T sr = vr[o], si = vi[o];
      for (int sl = 0; sl < it.j; ++sl) {
        const T *pr = p.num + p.part + (int64_t)(it.i + sl) * NB * mr * 2;
        const int64_t q = a + (int64_t)(j0 + j) * NB;
        sr -= pr[q];
        si -= pr[q + (int64_t)NB * mr];
      }
      zr[a][j] = sr;
      zi[a][j] = si;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < b * nj; e += 256) {
      const int a = e % b, j = e / b;
      T wr = zr[a][j], wi = zi[a][j];
      for (int c = a + 1; c < b; ++c) {
        const int64_t o = (k + c) + (int64_t)(k + a) * n;
        const T lr = fr[o], li = fi[o];
        wr += lr * zr[c][j] - li * zi[c][j];
        wi += lr * zi[c][j] + li * zr[c][j];
      }
      const int64_t o = k + pm[a] + (int64_t)(j0 + j) * n;
      vr[o] = wr;
      vi[o] = wi;
    }
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

// interface GEMV: mode 0: YG = X v_root ; mode 1: v_root = YG - X h
template <typename T>
__global__ __launch_bounds__(256) void k_gemv(KP<T> p, int mode, int nrhs) {
  __shared__ T redr[4][64][9], redi[4][64][9];
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
    T ar[8], ai[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) ar[q] = ai[q] = 0;
    if (r < g) {
      for (int c = cg; c < g; c += 4) {
        const int64_t o = r + (int64_t)c * g;
        const T xr = Xr[o], xi = Xi[o];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (j0 + q < nrhs) {
            const int64_t io = c + (int64_t)(j0 + q) * g;
            const T br = inr[io], bi = ini[io];
            ar[q] += xr * br - xi * bi;
            ai[q] += xr * bi + xi * br;
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
        if (j0 + q >= nrhs) break;
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
    __syncthreads();
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
// and per-block sums of |r|^2 (or |f|^2 when fnorm) per column
template <typename T>
__global__ __launch_bounds__(256) void k_r_resid(KP<T> p, const cd *f, int64_t ldf, int nrhs, int64_t part_off,
                                                 int fnorm) {
  __shared__ double red[256];
  const int64_t mr = p.mr;
  const double *U = p.r64;
  const double *L = U + 2 * p.n_torn * mr;
  double *part = p.r64 + part_off;
  const int64_t nrow = p.n_torn + p.n_mult;
  for (int j = 0; j < nrhs; ++j) {
    double acc = 0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nrow; e += (int64_t)gridDim.x * 256) {
      double rr, ri;
      if (e < p.n_torn) {
        const cd fv = f[e + j * ldf];
        rr = fv.re;
        ri = fv.im;
        if (!fnorm) {
          for (int64_t q = p.csrp[e]; q < p.csrp[e + 1]; ++q) {
            const cd a = p.vals[q];
            const int64_t c = p.csrc[q];
            const double ur = U[c + j * p.n_torn], ui = U[c + j * p.n_torn + p.n_torn * mr];
            rr -= a.re * ur - a.im * ui;
            ri -= a.re * ui + a.im * ur;
          }
          const int g = p.rowgam[e];
          if (g >= 0) {
            const GamRef G = p.grefs[g];
            for (int t = 0; t < G.cnt; ++t) {
              const int64_t m = p.hmult[G.beg + t];
              const double s = p.hsign[G.beg + t];
              rr -= s * L[m + j * p.n_mult];
              ri -= s * L[m + j * p.n_mult + p.n_mult * mr];
            }
          }
          T *vf = p.num + p.vf;
          vf[e + j * p.n_torn] = (T)rr;
          vf[e + j * p.n_torn + p.n_torn * mr] = (T)ri;
        }
      } else {
        if (fnorm) continue;
        const int64_t m = e - p.n_torn;
        const MultRef R = p.mrefs[m];
        rr = 0;
        ri = 0;
        for (int t = 0; t < 2; ++t) {
          const double s = R.sg[t];
          rr -= s * U[R.row[t] + j * p.n_torn];
          ri -= s * U[R.row[t] + j * p.n_torn + p.n_torn * mr];
        }
        T *vc = p.num + p.vc;
        vc[m + j * p.n_mult] = (T)rr;
        vc[m + j * p.n_mult + p.n_mult * mr] = (T)ri;
      }
      acc += rr * rr + ri * ri;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x + (int64_t)j * gridDim.x] = red[0];
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
      case L_INVPREP: hipLaunchKernelGGL(k_invprep<T>, g, b, 0, st, k, L.first); break;
      case L_INVTRMM: hipLaunchKernelGGL(k_invtrmm<T>, g, b, 0, st, k, L.first); break;
      case L_INVSYRK: hipLaunchKernelGGL(k_invsyrk<T>, g, b, 0, st, k, L.first); break;
      case S_FINIT: hipLaunchKernelGGL(k_finit<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_FDIAG: hipLaunchKernelGGL(k_fdiag<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_FUPD: hipLaunchKernelGGL(k_fupd<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_FFIN: hipLaunchKernelGGL(k_ffin<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_BINIT: hipLaunchKernelGGL(k_binit<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_BPART: hipLaunchKernelGGL(k_bpart<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_BDIAG: hipLaunchKernelGGL(k_bdiag<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_BFIN: hipLaunchKernelGGL(k_bfin<T>, g, b, 0, st, k, L.first, nrhs); break;
      default: return hipErrorInvalidValue;
    }
    if (timed) {
      (void)hipEventRecord(ev[tm->used + 1], st);
      tm->used += 2;
    }
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t factor_t(const Plan &P, uint8_t *ws, const void *vals, hipStream_t st, KTimer *tm) {
  KP<T> k = make_kp<T>(P, ws, vals);
  hipError_t e = hipMemsetAsync(k.status, 0, 2 * sizeof(int), st);
  if (e != hipSuccess) return e;
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
