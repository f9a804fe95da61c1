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
  const int32_t *urow;
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
  const int64_t *sellp;
  const int32_t *sellc;
  const int64_t *domrow;
  // subset solve: domains whose mask byte is 0 skip the backward
  // substitution (null: every domain)
  const uint8_t *dmask;
  const Item *gemv;
  // copies of each global DoF (FP64 refinement): representative torn row,
  // component pointers and rows
  const int32_t *grep;
  const int32_t *gcp;
  const int32_t *gcr;
  // refinement control: the kernels of a correction iteration return at
  // once when *skip is nonzero (the refinement has converged); null: ungated
  const int *skip;
  int64_t n_gcomp;
  int64_t rg;      // offset (doubles) of the assembled-residual rows in r64
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
  int32_t mr, n_dom;
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


// Output tile of the MFMA GEMMs: BM x BN, WR x WC waves, each wave owning an
// (XB*16) x (YB*16) block of 16 x 16 MFMA results.
// TK_ is the K depth of one LDS stage.
template <int BM_, int BN_, int WR_, int WC_, int TK_ = 16>
struct Tile {
  static constexpr int BM = BM_, BN = BN_, WR = WR_, WC = WC_, NTH = 64 * WR_ * WC_, TK = TK_;
  static constexpr int XB = BM_ / (16 * WR_), YB = BN_ / (16 * WC_);
  static constexpr int REPA = BM_ * TK_ / NTH, REPB = BN_ * TK_ / NTH;
  // Position of element i of result block (x, y): row (the m index) and
  // column (the c index) inside the tile.  The MFMA computes the transposed
  // block (first operand from B, second from A) so that the 16 lanes of a
  // result row run along m, the contiguous dimension of the column-major
  // tiles.  Its result row index is 4*(lane/16) + i for the FP32 instruction
  // and lane/16 + 4*i for the FP64 one; its column is lane%16.
  __device__ static __forceinline__ int row(int x) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    return (w / WC_) * (XB * 16) + x * 16 + (lane & 15);
  }
  template <typename T>
  __device__ static __forceinline__ int col(int y, int i) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int base = (w % WC_) * (YB * 16) + y * 16;
    if (sizeof(T) == 8) return base + (lane >> 4) + 4 * i;
    return base + (lane >> 4) * 4 + i;
  }
};
using T64 = Tile<64, 64, 2, 2>;      // 256 threads, 2 x 2 blocks per wave
// the same tile with 32-deep stages: half the dependent load / barrier steps
// for the short-K GEMMs on the pivot chain (column update, panel solve)
using T64K32 = Tile<64, 64, 2, 2, 32>;
using T128 = Tile<128, 128, 2, 4>;   // 512 threads, 4 x 2 blocks per wave

template <typename T, class TL>
struct alignas(16) GemmSmem {
  T a[2][TL::TK][TL::BM + 4];
  T b[2][TL::TK][TL::BN + 4];
};

// four consecutive elements from an address aligned to the element only
// (one or two dwordx4 loads)
typedef float f4u __attribute__((ext_vector_type(4))) __attribute__((aligned(4)));
typedef double d2u __attribute__((ext_vector_type(2))) __attribute__((aligned(8)));
__device__ __forceinline__ void load4(const float *p, float (&v)[4]) {
  const f4u x = *reinterpret_cast<const f4u *>(p);
  v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
}
__device__ __forceinline__ void load4(const double *p, double (&v)[4]) {
  const d2u x = reinterpret_cast<const d2u *>(p)[0], y = reinterpret_cast<const d2u *>(p)[1];
  v[0] = x.x; v[1] = x.y; v[2] = y.x; v[3] = y.y;
}

// elements x0 .. x0 + 3 of a column (planes pr / pi, element x at offset x):
// one vector load per plane when x0 + 3 < lim, else clamped to lim - 1 and
// zero from lim on (lim >= 1)
template <typename T>
__device__ __forceinline__ void col4(const T *pr, const T *pi, int x0, int lim, T (&re)[4], T (&im)[4]) {
  if (x0 + 3 < lim) {
    load4(pr + x0, re);
    load4(pi + x0, im);
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int x = min(x0 + e, lim - 1);
      const T a = pr[x], b = pi[x];
      re[e] = x0 + e < lim ? a : T(0);
      im[e] = x0 + e < lim ? b : T(0);
    }
  }
}

// Accumulates a BM x BN complex tile P = sum_k A(m,k) B(c,k) over k in
// [kbeg, kend).  fa(m, k, re, im) / fb(c, k, re, im) return operand values
// (and must leave zeros outside their valid range).  AK / BK select the
// thread mapping of the loads: true when the operand is contiguous along k.
// The next K chunk is fetched into registers while the current one is
// multiplied.  With VW = 4 (operands contiguous along m only) each thread
// fetches four consecutive m of one k: fa(m0, k, re[4], im[4]).
// G3 selects Gauss's three-product form of the complex product (Higham,
// "Stability of a method for multiplying complex matrices with three real
// matrix multiplications", SIMAX 1992): T1 = Ar Br, T2 = Ai Bi,
// T3 = (Ar + Ai)(Br + Bi), Re = T1 - T2, Im = T3 - T1 - T2.  It takes three
// matrix-core products per step instead of four and is stable normwise, not
// componentwise (the imaginary part can lose relative accuracy where it is
// small against |A||B|).
// VWB (default VW) sets the fetch width of the second operand on its own.
template <typename T, class TL, bool AK, bool BK, int VW = 1, bool G3 = false, int VWB = VW, class FA, class FB>
__device__ __forceinline__ void gemm_tile(GemmSmem<T, TL> &sm, int kbeg, int kend, FA fa, FB fb,
                                          typename V4<T>::t (&cr)[TL::XB][TL::YB],
                                          typename V4<T>::t (&ci)[TL::XB][TL::YB]) {
  constexpr int NTH = TL::NTH, XB = TL::XB, YB = TL::YB, RA = TL::REPA, RB = TL::REPB, TK = TL::TK;
  static_assert(VW == 1 || (VW == 4 && !AK && RA % 4 == 0), "vector fetch layout (first operand)");
  static_assert(VWB == 1 || (VWB == 4 && !BK && RB % 4 == 0), "vector fetch layout (second operand)");
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w / TL::WC, wc = w % TL::WC;
  typename V4<T>::t ct[XB][YB];   // T3 of the three-product form
#pragma unroll
  for (int x = 0; x < XB; ++x)
#pragma unroll
    for (int y = 0; y < YB; ++y) {
      cr[x][y] = typename V4<T>::t{0, 0, 0, 0};
      ci[x][y] = typename V4<T>::t{0, 0, 0, 0};
      ct[x][y] = typename V4<T>::t{0, 0, 0, 0};
    }
  // operand element `rep` of this thread: along k (contiguous) TK threads
  // cover one K chunk; otherwise BM (BN) threads cover one k
  auto ma_ = [&](int rep) { return AK ? tid / TK + (NTH / TK) * rep : tid % TL::BM; };
  auto ka_ = [&](int rep) { return AK ? tid % TK : tid / TL::BM + (NTH / TL::BM) * rep; };
  auto mb_ = [&](int rep) { return BK ? tid / TK + (NTH / TK) * rep : tid % TL::BN; };
  auto kb_ = [&](int rep) { return BK ? tid % TK : tid / TL::BN + (NTH / TL::BN) * rep; };
  T ra[2][RA], rb[2][RB];
  // vector layout: rep e of group g covers m = (tid % (BM/4)) * 4 + e at
  // k = tid / (BM/4) + (4 NTH / BM) g
  auto va_m = [&](int g) { return (tid % (TL::BM / 4)) * 4; };
  auto va_k = [&](int g) { return tid / (TL::BM / 4) + (4 * NTH / TL::BM) * g; };
  auto vb_m = [&](int g) { return (tid % (TL::BN / 4)) * 4; };
  auto vb_k = [&](int g) { return tid / (TL::BN / 4) + (4 * NTH / TL::BN) * g; };
  auto fetch = [&](int k0) {
    if constexpr (VW == 4) {
#pragma unroll
      for (int g = 0; g < RA / 4; ++g) {
        T re[4] = {0, 0, 0, 0}, im[4] = {0, 0, 0, 0};
        if (k0 + va_k(g) < kend) fa(va_m(g), k0 + va_k(g), re, im);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          ra[0][4 * g + e] = re[e];
          ra[1][4 * g + e] = im[e];
        }
      }
    } else {
#pragma unroll
      for (int rep = 0; rep < RA; ++rep) {
        const int m = ma_(rep), k = ka_(rep);
        T re = 0, im = 0;
        if (k0 + k < kend) fa(m, k0 + k, re, im);
        ra[0][rep] = re;
        ra[1][rep] = im;
      }
    }
    if constexpr (VWB == 4) {
#pragma unroll
      for (int g = 0; g < RB / 4; ++g) {
        T re[4] = {0, 0, 0, 0}, im[4] = {0, 0, 0, 0};
        if (k0 + vb_k(g) < kend) fb(vb_m(g), k0 + vb_k(g), re, im);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          rb[0][4 * g + e] = re[e];
          rb[1][4 * g + e] = im[e];
        }
      }
    } else {
#pragma unroll
      for (int rep = 0; rep < RB; ++rep) {
        const int m = mb_(rep), k = kb_(rep);
        T re = 0, im = 0;
        if (k0 + k < kend) fb(m, k0 + k, re, im);
        rb[0][rep] = re;
        rb[1][rep] = im;
      }
    }
  };
  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += TK) {
    __syncthreads();
    if constexpr (VW == 4) {
#pragma unroll
      for (int g = 0; g < RA / 4; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          sm.a[0][va_k(g)][va_m(g) + e] = ra[0][4 * g + e];
          sm.a[1][va_k(g)][va_m(g) + e] = ra[1][4 * g + e];
        }
    } else {
#pragma unroll
      for (int rep = 0; rep < RA; ++rep) {
        sm.a[0][ka_(rep)][ma_(rep)] = ra[0][rep];
        sm.a[1][ka_(rep)][ma_(rep)] = ra[1][rep];
      }
    }
    if constexpr (VWB == 4) {
#pragma unroll
      for (int g = 0; g < RB / 4; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          sm.b[0][vb_k(g)][vb_m(g) + e] = rb[0][4 * g + e];
          sm.b[1][vb_k(g)][vb_m(g) + e] = rb[1][4 * g + e];
        }
    } else {
#pragma unroll
      for (int rep = 0; rep < RB; ++rep) {
        sm.b[0][kb_(rep)][mb_(rep)] = rb[0][rep];
        sm.b[1][kb_(rep)][mb_(rep)] = rb[1][rep];
      }
    }
    __syncthreads();
    if (k0 + TK < kend) fetch(k0 + TK);
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const int kr = kk + (lane >> 4);
      T ar[XB], ai[XB], br[YB], bi[YB];
#pragma unroll
      for (int x = 0; x < XB; ++x) {
        ar[x] = sm.a[0][kr][wr * XB * 16 + x * 16 + (lane & 15)];
        ai[x] = sm.a[1][kr][wr * XB * 16 + x * 16 + (lane & 15)];
      }
#pragma unroll
      for (int y = 0; y < YB; ++y) {
        br[y] = sm.b[0][kr][wc * YB * 16 + y * 16 + (lane & 15)];
        bi[y] = sm.b[1][kr][wc * YB * 16 + y * 16 + (lane & 15)];
      }
      if constexpr (G3) {
        T as[XB], bs[YB];
#pragma unroll
        for (int x = 0; x < XB; ++x) as[x] = ar[x] + ai[x];
#pragma unroll
        for (int y = 0; y < YB; ++y) bs[y] = br[y] + bi[y];
#pragma unroll
        for (int x = 0; x < XB; ++x)
#pragma unroll
          for (int y = 0; y < YB; ++y) {
            cr[x][y] = mfma16(br[y], ar[x], cr[x][y]);
            ci[x][y] = mfma16(bi[y], ai[x], ci[x][y]);
            ct[x][y] = mfma16(bs[y], as[x], ct[x][y]);
          }
      } else {
#pragma unroll
        for (int x = 0; x < XB; ++x)
#pragma unroll
          for (int y = 0; y < YB; ++y) {
            cr[x][y] = mfma16(br[y], ar[x], cr[x][y]);
            cr[x][y] = mfma16(-bi[y], ai[x], cr[x][y]);
            ci[x][y] = mfma16(bi[y], ar[x], ci[x][y]);
            ci[x][y] = mfma16(br[y], ai[x], ci[x][y]);
          }
      }
    }
  }
  if constexpr (G3) {
#pragma unroll
    for (int x = 0; x < XB; ++x)
#pragma unroll
      for (int y = 0; y < YB; ++y) {
        const typename V4<T>::t t1 = cr[x][y], t2 = ci[x][y];
        cr[x][y] = t1 - t2;
        ci[x][y] = (ct[x][y] - t1) - t2;
      }
  }
}

// the 64 x 64 tile's output positions
__device__ __forceinline__ int out_row(int x) { return T64::row(x); }
template <typename T>
__device__ __forceinline__ int out_col(int y, int i) { return T64::col<T>(y, i); }

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
    // four columns per step; the loads are unconditional (a non-contributing
    // entry reads the child's update-block origin) and selected afterwards,
    // so all of a step's loads are in flight together
    const int cstop = min(cend, r + 1);
    for (int cb = c0; cb < cstop; cb += 4) {
      T vr[4] = {0, 0, 0, 0}, vi[4] = {0, 0, 0, 0};
#pragma unroll
      for (int ch = 0; ch < 8; ++ch) {
        if (ch >= ng) break;   // uniform
        T xr[4], xi[4];
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = cb + u;
          const int rcv = rmc[ch][min(c, cstop - 1) - c0];
          const int rc = c < cstop ? rcv : -1;
          ok[u] = rr[ch] >= 0 && rc >= 0;
          const int64_t o = coff[ch] + (ok[u] ? rr[ch] + rc * cn[ch] : 0);
          xr[u] = p.num[o];
          xi[u] = p.num[o + cplane[ch]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          vr[u] += ok[u] ? xr[u] : T(0);
          vi[u] += ok[u] ? xi[u] : T(0);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = cb + u;
        if (c >= cstop) break;
        const int64_t o = r + (int64_t)c * n;
        if (g0 == 0) {
          re[o] = vr[u];
          im[o] = vi[u];
        } else {
          re[o] += vr[u];
          im[o] += vi[u];
        }
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

// Auxiliary-front assembly: item (aux block pair, i0, j0) adds the 64 x 64
// sub-block of sum_d s s' X_d(gb, ga) at rows pb + j, columns pa + i.  Lanes
// run along j (contiguous front rows and interface positions); the four waves
// take every fourth i.
template <typename T>
__global__ __launch_bounds__(256) void k_auxg(KP<T> p, int64_t first) {
  const Item it = p.items[first + blockIdx.x];
  const AuxItem a = p.aux[it.f];
  const FrontDev f = p.F[a.f];
  T *re = p.num + f.off;
  T *im = re + (int64_t)f.n * f.n;
  const int j = it.j + (threadIdx.x & 63), ig = threadIdx.x >> 6;
  if (j >= a.nb) return;
  int64_t gb[2];
  int sb[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    gb[t] = t < a.ndom ? p.gpos[a.gb[t] + j] : 0;
    sb[t] = t < a.ndom ? p.gsign[a.gb[t] + j] : 0;
  }
  const int iend = min(it.i + 64, a.na);
  for (int i = it.i + ig; i < iend; i += 4) {
    if (a.same && j < i) continue;
    T sr = 0, si = 0;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      if (t < a.ndom) {
        const int64_t ga = p.gpos[a.ga[t] + i], g = a.g[t];
        const int sg = p.gsign[a.ga[t] + i] * sb[t];
        const T *X = p.num + a.xoff[t];
        const T xr = X[gb[t] + ga * g], xi = X[g * g + gb[t] + ga * g];
        sr += sg > 0 ? xr : -xr;
        si += sg > 0 ? xi : -xi;
      }
    }
    const int64_t o = (a.pb + j) + (int64_t)(a.pa + i) * f.n;
    re[o] += sr;
    im[o] += si;
  }
}

// Stored factor: columns [c0, c0 + 16) of front f on rows [r0, r0 + 256),
// from the full front matrix (ld n) to the stored-factor place (ld n,
// imaginary plane at loff + lpim), whose memory outlives the front.
template <typename T>
__global__ __launch_bounds__(256) void k_store(KP<T> p, int64_t first) {
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, r = it.i + threadIdx.x, c0 = it.k;
  if (r >= n) return;
  const int cend = min(c0 + 16, f.s);
  const T *sr = p.num + f.off;
  const T *si = sr + (int64_t)n * n;
  T *dr = p.num + f.loff;
  T *di = dr + f.lpim;
  T xr[16], xi[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int64_t o = r + (int64_t)min(c0 + u, cend - 1) * n;
    xr[u] = sr[o];
    xi[u] = si[o];
  }
#pragma unroll
  for (int u = 0; u < 16; ++u)
    if (c0 + u < cend) {
      const int64_t o = r + (int64_t)(c0 + u) * n;
      dr[o] = xr[u];
      di[o] = xi[u];
    }
}

// ---------------------------------------------------------------------------
// pivot tile: restricted Bunch-Kaufman LDL^T of the NB x NB diagonal tile in
// FP64, with L^-1 formed alongside (section II: pivot search confined to the
// diagonal block).
//
// The tile lives in registers, lane c of wave w holding column c, rows
// 16 w .. 16 w + 15 (four waves, one per SIMD), both triangles, in their
// original (physical) positions.  Interchanges are never carried out on the
// data: the order is a permutation kept per lane (positions pv, pos), and the
// active rows / columns are one 64-bit mask, uniform over the block.  One
// register set M serves both matrices: an active column holds the partially
// reduced tile A, an eliminated column the corresponding column of L^-1 (the
// two never need updating at the same entry; rows of eliminated pivots keep
// stale values in active columns, which are never read).
//
// A step publishes the pivot's row once: its owner wave writes its register of
// that row, one value per lane, in two forms (masked to the active columns
// other than the pivot: the pivot test and the multipliers of every wave's
// rows; raw with 1 at the pivot: the update row).  Every wave repeats the
// pivot test on it and updates all of its 16 x 64 entries as
// M(r, c) = keep(c) M(r, c) - cm(r) w(c), w = D^-1 z, keep = 0 on the pivot
// columns, which thereby become their columns of -L (of L^-1).  A step that
// keeps its diagonal pivot needs one barrier.  At most 128 registers, so that
// a workgroup is seated as soon as one workgroup of the trailing update that
// shares the CUs retires.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false),
                          __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false));
}
// maximum over the 64 lanes (DPP: quad swaps, half-row and row mirrors, then
// row broadcasts 15 and 31 accumulate into lane 63), returned in every lane
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0x141>(v));
  v = fmax(v, dpp_f64<0x140>(v));
  v = fmax(v, dpp_f64<0x142, 0xA>(v));
  v = fmax(v, dpp_f64<0x143, 0xC>(v));
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                          __builtin_amdgcn_readlane(__double2loint(v), 63));
}
// 1/x from the hardware reciprocal and one Newton step (a short dependency
// chain; x = 0 gives a non-finite result, which the callers test for)
__device__ __forceinline__ double rcp_nr(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

struct PanelSmem {
  double2 zrow[3][NB], cmrow[3][NB];   // published rows (buffers 0 / 1: next pivot, 2: candidate)
  double dgs[3][4];                    // their diagonal and its reciprocal
  double dvr[NB], dvi[NB], dor[NB], doi[NB];
  int pdl[NB];
  double red[4];
};

// Pivot tile of item it (tile columns [it.k, it.k + NB)).  pend: the tile's
// column update is pending in LDS (dst: 2 x NB rows of NB + 1, real parts
// then imaginary parts, lower triangle, in the front's precision) and is
// subtracted as the tile is loaded; ps may then overlay dst.
template <typename T>
__device__ __forceinline__ void panel_item(const KP<T> &p, const Item &it, PanelSmem &ps, const T (*dst)[NB + 1],
                                           bool pend) {
  double2 (&zrow)[3][NB] = ps.zrow;
  double2 (&cmrow)[3][NB] = ps.cmrow;
  double (&dgs)[3][4] = ps.dgs;
  double (&dvr)[NB] = ps.dvr;
  double (&dvi)[NB] = ps.dvi;
  double (&dor)[NB] = ps.dor;
  double (&doi)[NB] = ps.doi;
  int (&pdl)[NB] = ps.pdl;
  double (&red)[4] = ps.red;
  const FrontDev f = p.F[it.f];
  const int k = it.k, n = f.n, b = min(NB, f.s - k), tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r0 = 16 * w;   // first row of this wave
  T *fr = p.num + f.off;
  T *fi = fr + (int64_t)n * n;
  constexpr double ALPHA = 0.6403882032022076;   // (1 + sqrt(17)) / 8

  double mr[16], mi[16];
  double amax = 0;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int i = r0 + t;
    double xr = 0, xi = 0;
    if (i < b && lane < b) {
      const int hi = max(i, lane), lo = min(i, lane);
      const int64_t o = (k + hi) + (int64_t)(k + lo) * n;
      T ar = fr[o], ai = fi[o];
      if (pend) {
        ar -= dst[hi][lo];
        ai -= dst[NB + hi][lo];
      }
      xr = (double)ar;
      xi = (double)ai;
    }
    mr[t] = xr;
    mi[t] = xi;
    amax = fmax(amax, cabs1(xr, xi));
  }
  amax = wave_max(amax);
  if (pend) __syncthreads();   // every wave has read dst, which ps overlays
  if (lane == 0) red[w] = amax;

  unsigned long long act = b == 64 ? ~0ull : ((1ull << b) - 1);   // active physical rows / columns
  // row q (block-uniform) with values (xr, xi) in this lane's column, into
  // buffer s: masked to the active columns other than q, raw with 1 at q,
  // and the diagonal with its reciprocal
  auto put_row = [&](int q, int s, double xr, double xi) {
    const bool a = ((act >> lane) & 1) && lane != q;
    cmrow[s][lane] = a ? make_double2(xr, xi) : make_double2(0.0, 0.0);
    zrow[s][lane] = lane == q ? make_double2(1.0, 0.0) : make_double2(xr, xi);
    if (lane == q) {
      const double rd = rcp_nr(fma(xr, xr, xi * xi));
      dgs[s][0] = xr;
      dgs[s][1] = xi;
      dgs[s][2] = xr * rd;
      dgs[s][3] = -xi * rd;
    }
  };
  // register of row q in this wave, -1 if another wave holds it (uniform)
  auto slot_of = [&](int q) { return w == (q >> 4) ? (q & 15) : -1; };
  // publishes row q from registers: one uniform branch per register (no
  // dynamic register index)
  auto publish = [&](int q, int s) {
    const int qt = slot_of(q);
    if (qt < 0) return;
    // binary search over the register index (uniform branches)
    if (qt < 8) {
      if (qt < 4) {
        if (qt < 2) { if (qt == 0) put_row(q, s, mr[0], mi[0]); else put_row(q, s, mr[1], mi[1]); }
        else { if (qt == 2) put_row(q, s, mr[2], mi[2]); else put_row(q, s, mr[3], mi[3]); }
      } else {
        if (qt < 6) { if (qt == 4) put_row(q, s, mr[4], mi[4]); else put_row(q, s, mr[5], mi[5]); }
        else { if (qt == 6) put_row(q, s, mr[6], mi[6]); else put_row(q, s, mr[7], mi[7]); }
      }
    } else {
      if (qt < 12) {
        if (qt < 10) { if (qt == 8) put_row(q, s, mr[8], mi[8]); else put_row(q, s, mr[9], mi[9]); }
        else { if (qt == 10) put_row(q, s, mr[10], mi[10]); else put_row(q, s, mr[11], mi[11]); }
      } else {
        if (qt < 14) { if (qt == 12) put_row(q, s, mr[12], mi[12]); else put_row(q, s, mr[13], mi[13]); }
        else { if (qt == 14) put_row(q, s, mr[14], mi[14]); else put_row(q, s, mr[15], mi[15]); }
      }
    }
  };

  int pv = lane, pos = lane;   // physical index at position `lane`; position of physical `lane`
  int npert = 0, n2 = 0, nswap = 0;
  int j = 0, cur = 0;
  publish(0, 0);
  __syncthreads();
  const double tmax = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  const double tau = tmax > 0 ? 1e-12 * tmax : 1.0;

  while (j < b) {
    const int pj = __builtin_amdgcn_readlane(pv, j);
    double2 z = zrow[cur][lane];
    const double2 cmc = cmrow[cur][lane];
    double ir = dgs[cur][2], ii = dgs[cur][3];
    const double d0r = dgs[cur][0], d0i = dgs[cur][1];
    const double2 *cmp = cmrow[cur] + r0;   // multipliers of this wave's rows
    bool zpiv = d0r == 0.0 && d0i == 0.0;
    const double absakk = cabs1(d0r, d0i);
    const double cv = cabs1(cmc.x, cmc.y);   // 0 off the active rows and at pj
    int kind = 1, pp = pj, pm = pj;
    if (__ballot(absakk < ALPHA * cv)) {
      const double colmax = wave_max(cv);
      pm = __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)__ballot(cv == colmax)) - 1);
      pm = pm < 0 ? pj : pm;   // (a lane attains the maximum unless the values are not finite)
      publish(pm, 2);
      __syncthreads();
      const double2 c2 = cmrow[2][lane];
      const double rowmax = wave_max(cabs1(c2.x, c2.y));
      const double e0 = dgs[2][0], e1 = dgs[2][1];
      if (absakk * rowmax >= ALPHA * colmax * colmax) {
        kind = 1;
      } else if (cabs1(e0, e1) >= ALPHA * rowmax) {
        kind = 1;
        pp = pm;
      } else {
        kind = 2;
      }
      kind = __builtin_amdgcn_readfirstlane(kind);
      pp = __builtin_amdgcn_readfirstlane(pp);
      if (kind == 2 || pp == pm) {
        // interchange of positions q and that of pm: only the order changes
        const int q = kind == 1 ? j : j + 1;
        const int ip = __builtin_amdgcn_readlane(pos, pm);
        if (ip != q) {
          const int a0 = __builtin_amdgcn_readlane(pv, q);
          pv = lane == q ? pm : (lane == ip ? a0 : pv);
          pos = lane == pm ? q : (lane == a0 ? ip : pos);
          ++nswap;
        }
      }
      if (kind == 1 && pp == pm) {
        cmp = cmrow[2] + r0;
        z = zrow[2][lane];
        ir = dgs[2][2];
        ii = dgs[2][3];
        zpiv = e0 == 0.0 && e1 == 0.0;
      }
      if (kind == 2) {
        // the two pivot rows take no update: clear pm's multiplier in pj's
        // row and pj's in pm's (every wave has read its test values)
        if (tid == 0) {
          cmrow[cur][pm] = make_double2(0.0, 0.0);
          cmrow[2][pj] = make_double2(0.0, 0.0);
        }
        __syncthreads();
      }
    }
    // the update, one pass per pivot row: M(r, c) = keep(c) M(r, c) - cm(r) w(c)
    const double2 *cmb = cmrow[2] + r0;   // second pass: the second row of a 2 x 2 pivot
    double wr, wi, w2r = 0, w2i = 0, keep;
    int npass = 1;
    if (kind == 1) {
      if (zpiv) {
        ir = 1.0 / tau;
        ii = 0.0;
        ++npert;
      }
      if (tid == 0) {
        dvr[j] = ir; dvi[j] = ii; dor[j] = 0; doi[j] = 0; pdl[j] = 0;
      }
      wr = z.x * ir - z.y * ii;
      wi = z.x * ii + z.y * ir;
      keep = lane == pp ? 0.0 : 1.0;
      act &= ~(1ull << pp);
      j += 1;
    } else {
      // 2 x 2 pivot (pj, pm) at positions j, j + 1
      const double2 zc = zrow[cur][lane], zm = zrow[2][lane];
      double ar_ = d0r, ai_ = d0i;
      const double2 cc = zrow[cur][pm];
      const double cr_ = cc.x, ci_ = cc.y;
      double er_ = dgs[2][0], ei_ = dgs[2][1];
      double detr = (ar_ * er_ - ai_ * ei_) - (cr_ * cr_ - ci_ * ci_);
      double deti = (ar_ * ei_ + ai_ * er_) - 2.0 * cr_ * ci_;
      if (detr == 0.0 && deti == 0.0) {
        ar_ += tau;
        er_ += tau;
        detr = (ar_ * er_ - ai_ * ei_) - (cr_ * cr_ - ci_ * ci_);
        deti = (ar_ * ei_ + ai_ * er_) - 2.0 * cr_ * ci_;
        ++npert;
      }
      const double rden = rcp_nr(fma(detr, detr, deti * deti));
      const double idr = detr * rden, idi = -deti * rden;
      const double d00r = er_ * idr - ei_ * idi, d00i = er_ * idi + ei_ * idr;
      const double d11r = ar_ * idr - ai_ * idi, d11i = ar_ * idi + ai_ * idr;
      const double d01r = -(cr_ * idr - ci_ * idi), d01i = -(cr_ * idi + ci_ * idr);
      if (tid == 0) {
        dvr[j] = d00r; dvi[j] = d00i; dvr[j + 1] = d11r; dvi[j + 1] = d11i;
        dor[j] = d01r; doi[j] = d01i; dor[j + 1] = d01r; doi[j + 1] = d01i;
        pdl[j] = 1; pdl[j + 1] = -1;
      }
      // update rows z0 (pj's, 0 at pm) and z1 (pm's, 0 at pj), [w w2] = D^-1 [z0 z1]
      const double z0r = lane == pm ? 0.0 : zc.x, z0i = lane == pm ? 0.0 : zc.y;
      const double z1r = lane == pj ? 0.0 : zm.x, z1i = lane == pj ? 0.0 : zm.y;
      wr = (d00r * z0r - d00i * z0i) + (d01r * z1r - d01i * z1i);
      wi = (d00r * z0i + d00i * z0r) + (d01r * z1i + d01i * z1r);
      w2r = (d01r * z0r - d01i * z0i) + (d11r * z1r - d11i * z1i);
      w2i = (d01r * z0i + d01i * z0r) + (d11r * z1i + d11i * z1r);
      keep = (lane == pj || lane == pm) ? 0.0 : 1.0;
      act &= ~((1ull << pj) | (1ull << pm));
      ++n2;
      j += 2;
      npass = 2;
    }
    for (int ps = 0; ps < npass; ++ps) {
      // multipliers of the wave's rows (broadcast reads), four at a time,
      // the next four in flight
      double2 ca[4], cb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) ca[u] = cmp[u];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        if (g < 3) {
#pragma unroll
          for (int u = 0; u < 4; ++u) cb[u] = cmp[4 * g + 4 + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int t = 4 * g + u;
          const double tr = fma(ca[u].x, wr, -ca[u].y * wi), ti = fma(ca[u].x, wi, ca[u].y * wr);
          mr[t] = fma(mr[t], keep, -tr);
          mi[t] = fma(mi[t], keep, -ti);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) ca[u] = cb[u];
      }
      cmp = cmb;
      wr = w2r;
      wi = w2i;
      keep = 1.0;
    }
    if (j < b) publish(__builtin_amdgcn_readlane(pv, j), cur ^ 1);
    cur ^= 1;
    __syncthreads();
  }
  // L^-1 in the pivoted order into the strict lower triangle of the tile:
  // position (a, c) is physical (pv[a], pv[c])
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int a = __builtin_amdgcn_readlane(pos, r0 + t);
    if (r0 + t < b && lane < b && pos < a) {
      const int64_t o = (k + a) + (int64_t)(k + pos) * n;
      fr[o] = (T)mr[t];
      fi[o] = (T)mi[t];
    }
  }
  bool bad = false;
  if (tid < b) {
    const int64_t s = f.soff + k + tid;
    p.dinv[s] = cd{dvr[tid], dvi[tid]};
    p.doff[s] = cd{dor[tid], doi[tid]};
    p.pdel[s] = pdl[tid];
    p.perm[s] = pv;
    if (!isfinite(dvr[tid]) || !isfinite(dvi[tid])) bad = true;
  }
  const int where = f.dom >= 0 ? f.dom : p.n_dom;
  if (bad) {
    atomicOr(p.status + 1, 1);
    atomicMin(p.status + 4, where);
  }
  if (tid == 0) {
    if (npert) {
      atomicAdd(p.status, npert);
      atomicMin(p.status + 4, where);
    }
    if (n2) atomicAdd(p.status + 2, n2);
    if (nswap) atomicAdd(p.status + 3, nswap);
  }
}

template <typename T>
__global__ __launch_bounds__(256, 4) void k_panel(KP<T> p, int64_t first) {
  __shared__ PanelSmem ps;
  panel_item<T>(p, p.items[first + blockIdx.x], ps, nullptr, false);
}

// W = A21 P^T L11^-T (rows r0..r0+GT), L21 = W D^-1
// At most 128 registers (four waves per SIMD) and, in FP64, 16-deep K
// stages (35 KB of LDS): while the side stream's Schur update fills the CUs
// (FP32: five 96-register workgroups per SIMD; FP64: four 128-register, 35 KB
// workgroups per CU), a workgroup of this size is seated as soon as one of
// them retires; larger ones wait until the update has no workgroups left to
// hand out.  The W tile is staged in the GEMM's LDS for the D^-1 step, in
// FP64 in two column halves (with the neighbouring column of each, the other
// row of a 2 x 2 pivot).
template <typename T>
__global__ __launch_bounds__(256, 4) void k_trsm(KP<T> p, int64_t first) {
  using TL = typename std::conditional<sizeof(T) == 8, T64, T64K32>::type;
  constexpr int HC = sizeof(T) == 8 ? 32 : GT;   // columns per staged part
  constexpr int WS = HC + 2;                     // with one column on each side
  __shared__ GemmSmem<T, TL> sm;
  static_assert(2 * GT * WS * sizeof(T) <= sizeof(GemmSmem<T, TL>), "W staging in the GEMM LDS");
  T(*wr)[WS] = reinterpret_cast<T(*)[WS]>(&sm.a[0][0][0]);
  T(*wi)[WS] = wr + GT;
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int k = it.k, r0 = it.i, n = f.n, b = min(NB, f.s - k);
  T *fr = p.num + f.off;
  T *fi = fr + (int64_t)n * n;
  const int32_t *pm = p.perm + f.soff + k;
  // four consecutive rows of one column (vector loads, clamped tails)
  auto fa = [&](int m, int kk, T (&re)[4], T (&im)[4]) {
    if (kk < b) {
      const int64_t col = (int64_t)(k + pm[kk]) * n;
      col4(fr + col, fi + col, r0 + m, n, re, im);
    }
  };
  // L11^-1 (unit lower, stored strictly below the diagonal): entries
  // (c .. c+3, kk) of the tile
  auto fb = [&](int c, int kk, T (&re)[4], T (&im)[4]) {
    const int64_t col = k + (int64_t)(k + kk) * n;
    col4(fr + col, fi + col, c, b, re, im);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const bool below = kk < c + e;
      re[e] = below ? re[e] : (kk == c + e && c + e < b ? T(1) : T(0));
      im[e] = below ? im[e] : T(0);
    }
  };
  typename V4<T>::t cr[2][2], ci[2][2];
  gemm_tile<T, TL, false, false, 4>(sm, 0, b, fa, fb, cr, ci);
  // W buffer of the outer block starting at k - it.j
  T *Wr = p.num + f.woff + (((k - it.j) / KBLK) & 1) * f.wstride;
  T *Wi = Wr + (int64_t)n * f.wcols;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = out_row(x), c = out_col<T>(y, i);
        if (r0 + m < n && c < b) {
          Wr[(r0 + m) + (int64_t)(it.j + c) * n] = cr[x][y][i];
          Wi[(r0 + m) + (int64_t)(it.j + c) * n] = ci[x][y][i];
        }
      }
  for (int c0 = 0; c0 < b; c0 += HC) {
    __syncthreads();   // every wave is done with the GEMM's LDS / the previous part
    // columns [c0 - 1, c0 + HC + 1) of the tile at wr[m][c - c0 + 1]
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = out_row(x), c = out_col<T>(y, i), cl = c - c0 + 1;
          if (cl >= 0 && cl < WS) {
            wr[m][cl] = cr[x][y][i];
            wi[m][cl] = ci[x][y][i];
          }
        }
    __syncthreads();
    const int ce = min(b, c0 + HC);
    for (int e = threadIdx.x; e < GT * (ce - c0); e += 256) {
      const int m = e % GT, c = c0 + e / GT, r = r0 + m, cl = c - c0 + 1;
      if (r >= n) continue;
      const int64_t s = f.soff + k + c;
      const cd d = p.dinv[s];
      double xr = (double)wr[m][cl] * d.re - (double)wi[m][cl] * d.im;
      double xi = (double)wr[m][cl] * d.im + (double)wi[m][cl] * d.re;
      const int pd = p.pdel[s];
      if (pd) {
        const cd o = p.doff[s];
        const double yr = (double)wr[m][cl + pd], yi = (double)wi[m][cl + pd];
        xr += yr * o.re - yi * o.im;
        xi += yr * o.im + yi * o.re;
      }
      fr[r + (int64_t)(k + c) * n] = (T)xr;
      fi[r + (int64_t)(k + c) * n] = (T)xi;
    }
  }
}

// Update of the trailing part by the factored columns [k, kend) of the current
// outer block: C(r0.., q0..) -= L21(r0.., k..kend) W(q0.., 0..kend-k)^T.
// Trailing update (q0 >= block end): lower tiles of the trailing matrix,
// kend = min(k + KBLK, s).  Column update (q0 < block end): the pivot tile
// column starting at q0 receives the block's earlier tiles, kend = q0.
// G3: Gauss's three-product form of the complex product.
template <typename T, class TL, bool G3 = (sizeof(T) == 4)>
__device__ __forceinline__ void syrk_item(const KP<T> &p, const Item &it, GemmSmem<T, TL> &sm) {
  const FrontDev f = p.F[it.f];
  const int k = it.k, r0 = it.i, q0 = it.j, n = f.n;
  const int bend = min(k + KBLK, f.s);
  const bool colupd = q0 < bend;
  const int kend = colupd ? q0 : bend;
  const int qend = colupd ? min(q0 + NB, f.s) : n;
  T *fr = p.num + f.off;
  T *fi = fr + (int64_t)n * n;
  const T *Wr = p.num + f.woff + ((k / KBLK) & 1) * f.wstride;   // the outer block's W buffer
  const T *Wi = Wr + (int64_t)n * f.wcols;
  // four consecutive rows of a column: one vector load each plane when all
  // four are in range
  auto fa = [&](int m, int kk, T (&re)[4], T (&im)[4]) {
    const int r = r0 + m;
    const int64_t o = r + (int64_t)kk * n;
    if (r + 3 < n) {
      load4(fr + o, re);
      load4(fi + o, im);
    } else {
      // clamped rows, selected afterwards (no per-element branches)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t oe = min(r + e, n - 1) + (int64_t)kk * n;
        const T xr = fr[oe], xi = fi[oe];
        re[e] = r + e < n ? xr : T(0);
        im[e] = r + e < n ? xi : T(0);
      }
    }
  };
  auto fb = [&](int c, int kk, T (&re)[4], T (&im)[4]) {
    const int q = q0 + c;
    const int64_t o = q + (int64_t)(kk - k) * n;
    if (q + 3 < qend) {
      load4(Wr + o, re);
      load4(Wi + o, im);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t oe = min(q + e, qend - 1) + (int64_t)(kk - k) * n;
        const T xr = Wr[oe], xi = Wi[oe];
        re[e] = q + e < qend ? xr : T(0);
        im[e] = q + e < qend ? xi : T(0);
      }
    }
  };
  typename V4<T>::t cr[TL::XB][TL::YB], ci[TL::XB][TL::YB];
  // G3: set for the trailing update (both precisions) and for the pivot
  // chain's column update in FP32; the panel solve keeps four products.
  gemm_tile<T, TL, false, false, 4, G3>(sm, k, kend, fa, fb, cr, ci);
  const bool diag = (r0 == q0);
#pragma unroll
  for (int x = 0; x < TL::XB; ++x)
#pragma unroll
    for (int y = 0; y < TL::YB; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = TL::row(x), c = TL::template col<T>(y, i);
        const int r = r0 + m, q = q0 + c;
        if (r < n && q < qend && (!diag || m >= c)) {
          const int64_t o = r + (int64_t)q * n;
          fr[o] -= cr[x][y][i];
          fi[o] -= ci[x][y][i];
        }
      }
}

// The trailing update runs the three-product form in both precisions.
// 64-edge tiles ask for four waves per SIMD in FP32 (96 registers) and three
// in FP64 (at most 168: the third accumulator set), so that one retiring
// workgroup seats a 128-register workgroup of the pivot chain.
template <typename T, class TL>
__global__ __launch_bounds__(TL::NTH, TL::BM == 64 ? (sizeof(T) == 8 ? 3 : 4) : 1) void k_syrk(KP<T> p,
                                                                                              int64_t first) {
  __shared__ GemmSmem<T, TL> sm;
  syrk_item<T, TL, true>(p, p.items[first + blockIdx.x], sm);
}

// Column update and pivot tile in one launch.  A pivot tile needs only the
// diagonal block of its column update, so its workgroup computes that block
// itself (the column update's product, staged in LDS) and factors the tile,
// while the other workgroups update the rows below: the pivot chain no longer
// waits for the whole column update.  Items {f, k, -1, o}: pivot tile k of
// front f in the outer block starting at o; other items: column-update items
// (rows below the diagonal block).
template <typename T>
__global__ __launch_bounds__(256, 4) void k_updpanel(KP<T> p, int64_t first) {
  // FP64: 16-deep K stages (35 KB of LDS, like the side stream's update
  // workgroups, so that one retirement seats a workgroup), and the diagonal
  // block goes through the front instead of a 66 KB LDS stage
  using TL = typename std::conditional<sizeof(T) == 8, T64, T64K32>::type;
  constexpr bool STAGE = sizeof(T) == 4;
  static_assert(sizeof(PanelSmem) <= sizeof(GemmSmem<T, TL>), "pivot-tile LDS inside the GEMM LDS");
  static_assert(!STAGE || 2 * NB * (NB + 1) * sizeof(T) <= sizeof(GemmSmem<T, TL>), "staged block in the GEMM LDS");
  __shared__ GemmSmem<T, TL> sm;
  const Item it = p.items[first + blockIdx.x];
  if (it.i >= 0) {
    syrk_item<T, TL>(p, it, sm);
    return;
  }
  const FrontDev f = p.F[it.f];
  const int k = it.k, o = it.j, n = f.n, s = f.s, b = min(NB, s - k);
  T *fr = p.num + f.off;
  T *fi = fr + (int64_t)n * n;
  const T *Wr = p.num + f.woff + ((o / KBLK) & 1) * f.wstride;   // the outer block's W buffer
  const T *Wi = Wr + (int64_t)n * f.wcols;
  // the column update's operands for rows [k, k + NB) and columns [k, k + b)
  auto fa = [&](int m, int kk, T (&re)[4], T (&im)[4]) {
    const int r = k + m;
    const int64_t x = r + (int64_t)kk * n;
    if (r + 3 < n) {
      load4(fr + x, re);
      load4(fi + x, im);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t xe = min(r + e, n - 1) + (int64_t)kk * n;
        const T vr = fr[xe], vi = fi[xe];
        re[e] = r + e < n ? vr : T(0);
        im[e] = r + e < n ? vi : T(0);
      }
    }
  };
  auto fb = [&](int c, int kk, T (&re)[4], T (&im)[4]) {
    const int q = k + c;
    const int64_t x = q + (int64_t)(kk - o) * n;
    if (q + 3 < k + b) {
      load4(Wr + x, re);
      load4(Wi + x, im);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t xe = min(q + e, k + b - 1) + (int64_t)(kk - o) * n;
        const T vr = Wr[xe], vi = Wi[xe];
        re[e] = q + e < k + b ? vr : T(0);
        im[e] = q + e < k + b ? vi : T(0);
      }
    }
  };
  typename V4<T>::t cr[TL::XB][TL::YB], ci[TL::XB][TL::YB];
  gemm_tile<T, TL, false, false, 4, sizeof(T) == 4>(sm, o, k, fa, fb, cr, ci);
  if (!STAGE) {
    // the column update of the block's lower triangle, as the column update
    // writes it; the tile is then loaded from the front (visible to the
    // workgroup after the barrier)
#pragma unroll
    for (int x = 0; x < TL::XB; ++x)
#pragma unroll
      for (int y = 0; y < TL::YB; ++y)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = TL::row(x), c = TL::template col<T>(y, i);
          if (c < b && m >= c && k + m < n) {
            const int64_t e = (k + m) + (int64_t)(k + c) * n;
            fr[e] -= cr[x][y][i];
            fi[e] -= ci[x][y][i];
          }
        }
    __syncthreads();
    panel_item<T>(p, it, *reinterpret_cast<PanelSmem *>(&sm), nullptr, false);
    return;
  }
  __syncthreads();   // every wave is done with the GEMM's LDS
  T(*dst)[NB + 1] = reinterpret_cast<T(*)[NB + 1]>(&sm);
#pragma unroll
  for (int x = 0; x < TL::XB; ++x)
#pragma unroll
    for (int y = 0; y < TL::YB; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = TL::row(x), c = TL::template col<T>(y, i);
        if (c < b && m >= c) {
          if (m < b) {
            dst[m][c] = cr[x][y][i];
            dst[NB + m][c] = ci[x][y][i];
          } else if (k + m < n) {
            // rows past the last pivot tile's end (update rows): as the
            // column update writes them
            const int64_t e = (k + m) + (int64_t)(k + c) * n;
            fr[e] -= cr[x][y][i];
            fi[e] -= ci[x][y][i];
          }
        }
      }
  __syncthreads();
  panel_item<T>(p, it, *reinterpret_cast<PanelSmem *>(&sm), dst, true);
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
// Both products take the three-product complex form (FP64 at two waves per
// SIMD: at three its accumulators would spill).
// The row block is one pivot tile (r0 is a multiple of the tile size): the
// product runs over the stored rows (contiguous, 16-byte loads) and each
// result row is written to its true row, found from the tile's permutation
// inverted in LDS.
// three waves per SIMD in FP32, two in FP64 (no spills at those budgets)
template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 8 ? 2 : 3) void k_zrec1(KP<T> p, int64_t first) {
  __shared__ GemmSmem<T, T64> sm;
  __shared__ int tr_of[NB];   // stored row r0 + i holds true row r0 + tr_of[i]
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int m0 = it.k, r0 = it.i, c0 = it.j, n = f.n, s = f.s;
  T *fr = p.num + f.off;
  T *fi = fr + (int64_t)n * n;
  const int32_t *pm = p.perm + f.soff;
  static_assert(GT == NB, "row blocks are pivot tiles");
  if (threadIdx.x < NB && r0 + (int)threadIdx.x < s) tr_of[pm[r0 + threadIdx.x]] = threadIdx.x;
  // stored rows r0 + m .. + 3 of column kk (zero from s on)
  auto fa = [&](int m, int kk, T (&re)[4], T (&im)[4]) {
    const int64_t col = (int64_t)kk * n;
    col4(fr + col, fi + col, r0 + m, s, re, im);
  };
  auto fb = [&](int c, int kk, T &re, T &im) {   // Z(kk, c0 + c)
    zval(fr, fi, n, kk, c0 + c, re, im);
  };
  typename V4<T>::t cr[2][2], ci[2][2];
  gemm_tile<T, T64, false, true, 4, true, 1>(sm, c0, m0, fa, fb, cr, ci);
  __syncthreads();   // tr_of complete (also for an empty K range)
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = out_row(x), c = out_col<T>(y, i);
        if (r0 + m < s && c0 + c < m0) {
          const int64_t o = (c0 + c) + (int64_t)(r0 + tr_of[m]) * n;
          fr[o] = cr[x][y][i];
          fi[o] = ci[x][y][i];
        }
      }
}

// three waves per SIMD in FP32, two in FP64 (no spills at those budgets)
template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 8 ? 2 : 3) void k_zrec2(KP<T> p, int64_t first) {
  __shared__ GemmSmem<T, T64> sm;
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int m0 = it.k, r0 = it.i, c0 = it.j, n = f.n, s = f.s;
  T *fr = p.num + f.off;
  T *fi = fr + (int64_t)n * n;
  auto fa = [&](int m, int kk, T (&re)[4], T (&im)[4]) {   // Z(r0 + m .. + 3, kk)
    const int r = r0 + m;
    const int64_t col = (int64_t)kk * n;
    col4(fr + col, fi + col, r, s, re, im);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const bool below = r + e > kk;
      re[e] = below ? re[e] : (r + e == kk && r + e < s ? T(1) : T(0));
      im[e] = below ? im[e] : T(0);
    }
  };
  auto fb = [&](int c, int kk, T (&re)[4], T (&im)[4]) {   // T1(kk, c0 + c ..), stored at (c0 + c .., kk)
    const int64_t col = (int64_t)kk * n;
    col4(fr + col, fi + col, c0 + c, m0, re, im);
  };
  typename V4<T>::t cr[2][2], ci[2][2];
  gemm_tile<T, T64, false, false, 4, true>(sm, m0, min(r0 + GT, s), fa, fb, cr, ci);
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

// Y = D^-1 Z of an interface root: the 1 x 1 and 2 x 2 pivots applied to the
// rows of Z = L^-1 (FP64 arithmetic, rounded to the front type).  Once Z is
// complete the front's diagonal and upper triangle are free (Z is unit lower,
// D is kept apart), so Y is stored there transposed: Y(r, c), r >= c, at
// position (c, r).  The only entries of Y above its diagonal, Y(r - 1, r) of
// a 2 x 2 pivot (r - 1, r), equal its off-diagonal D^-1 entry and are not
// stored.  Item (f, 0, r0, c0), r0 >= c0: the 64 x 64 tile rows
// [r0, r0 + 64) x columns [c0, c0 + 64) of Y, transposed through LDS so that
// both the reads of Z and the writes of Y^T run along contiguous rows.  Reads
// touch only the strict lower triangle and writes only the rest, so the
// tiles are independent.
template <typename T>
__global__ __launch_bounds__(256) void k_dinvz(KP<T> p, int64_t first) {
  __shared__ T yr_[64][65], yi_[64][65];
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, r0 = it.i, c0 = it.j, tid = threadIdx.x;
  T *fr = p.num + f.off;
  T *fi = fr + (int64_t)n * n;
  const cd *dv = p.dinv + f.soff;
  const cd *dof = p.doff + f.soff;
  const int32_t *pd = p.pdel + f.soff;
#pragma unroll 4
  for (int u = 0; u < 16; ++u) {
    const int rr = tid & 63, cc = (tid >> 6) + 4 * u, r = r0 + rr, c = c0 + cc;
    double xr = 0, xi = 0;
    if (r < n && c < n && r >= c) {
      T zr = 0, zi = 0;
      zval(fr, fi, n, r, c, zr, zi);
      const cd d = dv[r];
      xr = d.re * (double)zr - d.im * (double)zi;
      xi = d.re * (double)zi + d.im * (double)zr;
      const int q = pd[r];
      if (q) {
        T wr = 0, wi = 0;
        zval(fr, fi, n, r + q, c, wr, wi);
        const cd o = dof[r];
        xr += o.re * (double)wr - o.im * (double)wi;
        xi += o.re * (double)wi + o.im * (double)wr;
      }
    }
    yr_[cc][rr] = (T)xr;
    yi_[cc][rr] = (T)xi;
  }
  __syncthreads();
#pragma unroll 4
  for (int u = 0; u < 16; ++u) {
    const int cc = tid & 63, rr = (tid >> 6) + 4 * u, r = r0 + rr, c = c0 + cc;
    if (r < n && c < n && r >= c) {
      const int64_t o = c + (int64_t)r * n;
      fr[o] = yr_[cc][rr];
      fi[o] = yi_[cc][rr];
    }
  }
}

// X(P a, P c) = sum_r Z(r, a) Y(r, c), Y = D^-1 Z as stored by k_dinvz;
// lower tiles, written to both triangles; three-product complex form (two
// waves per SIMD in FP64, whose 2 x 2 accumulator sets need the registers)
template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 8 ? 2 : 3) void k_invsyrk(KP<T> p, int64_t first) {
  __shared__ GemmSmem<T, T64> sm;
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int a0 = it.i, c0 = it.j, n = f.n;
  const T *fr = p.num + f.off;
  const T *fi = fr + (int64_t)n * n;
  const cd *dof = p.doff + f.soff;
  const int32_t *pd = p.pdel + f.soff;
  const int32_t *pm = p.perm + f.soff;
  auto fa = [&](int m, int kk, T &re, T &im) {
    const int a = a0 + m;
    if (a < n) zval(fr, fi, n, kk, a, re, im);
  };
  // Y(kk, c0 + c): Y^T row c0 + c, contiguous along c
  auto fb = [&](int c, int kk, T &re, T &im) {
    const int cc = c0 + c;
    if (cc >= n) return;
    if (kk >= cc) {
      const int64_t o = cc + (int64_t)kk * n;
      re = fr[o];
      im = fi[o];
    } else if (kk == cc - 1 && pd[kk] == 1) {
      const cd o = dof[kk];
      re = (T)o.re;
      im = (T)o.im;
    }
  };
  typename V4<T>::t cr[2][2], ci[2][2];
  gemm_tile<T, T64, true, false, 1, true>(sm, a0, n, fa, fb, cr, ci);
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

// subset solve: is front f's domain left out of the backward substitution?
template <typename T>
__device__ __forceinline__ bool skipped(const KP<T> &p, const FrontDev &f) {
  return p.dmask && f.dom >= 0 && !p.dmask[f.dom];
}
// a converged refinement skips the rest of its enqueued iterations
template <typename T>
__device__ __forceinline__ bool gated(const KP<T> &p) {
  return p.skip && *(volatile const int *)p.skip != 0;
}

// Row-by-column split of a workgroup over `live` rows of a front vector: the
// smallest power of two R >= live (at least 8, at most cap) takes the rows, and
// the workgroup's other threads take further right-hand-side columns (thread
// t: row t mod R, columns t / R, t / R + G, ... with G = threads / R), so the
// small fronts of the lower levels keep the whole workgroup busy.
struct RowSplit {
  int r, g, G, sh;   // row offset, first column, column stride, log2(R)
};
__device__ __forceinline__ RowSplit row_split(int live, int cap, int threads) {
  int sh = 3;
  while ((1 << sh) < live && (1 << sh) < cap) ++sh;
  const int t = threadIdx.x;
  return RowSplit{t & ((1 << sh) - 1), t >> sh, threads >> sh, sh};
}

// ---------------------------------------------------------------------------
// multi-RHS substitutions (front vectors v: n x mr planar, ld n)
// Front vector rows [it.i, it.i + 256): gathered right-hand side on the
// fully-summed rows plus the children's update parts (extend-add).  A front
// without children gets its fully-summed rows only: its forward product
// writes the update rows outright.
template <typename T>
__global__ __launch_bounds__(256) void k_finit(KP<T> p, int64_t first, int nrhs) {
  if (gated(p)) return;
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, s = f.s, hi = f.nchild ? n : s;
  const RowSplit rs = row_split(min(256, hi - it.i), 256, 256);
  const int r = it.i + rs.r, G = rs.G;
  if (r >= hi) return;
  const int64_t mr = p.mr;
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)n * mr;
  const bool aux = f.kind == FK_AUX;
  const int64_t ld = aux ? p.n_mult : p.n_torn;
  const T *sr = p.num + (aux ? p.vd : p.vf);
  const T *si = sr + ld * mr;
  const int64_t row = r < s ? f.vbase + p.vars[f.idx + r] : -1;
  // children that contribute to row r (up to 8 in registers; the rest, if
  // any, are added in a second pass)
  const T *cp[8];
  int cn[8];
  int nc = 0, ch = 0;
  for (; ch < f.nchild && nc < 8; ++ch) {
    const int rr = p.rmap[p.crmap[f.child + ch] + r];
    if (rr < 0) continue;
    const FrontDev &cf = p.F[p.cfront[f.child + ch]];
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (c == nc) {
        cp[c] = p.num + cf.voff + cf.s + rr;
        cn[c] = cf.n;
      }
    ++nc;
  }
  // eight of this thread's right-hand sides at a time: all loads, then the
  // stores
  for (int j0 = rs.g; j0 < nrhs; j0 += 8 * G) {
    T xr[8], xi[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int j = min(j0 + q * G, nrhs - 1);
      xr[q] = row >= 0 ? sr[row + (int64_t)j * ld] : T(0);
      xi[q] = row >= 0 ? si[row + (int64_t)j * ld] : T(0);
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (c >= nc) break;
      const int64_t pl = (int64_t)cn[c] * mr;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int j = min(j0 + q * G, nrhs - 1);
        xr[q] += cp[c][(int64_t)j * cn[c]];
        xi[q] += cp[c][(int64_t)j * cn[c] + pl];
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (j0 + q * G < nrhs) {
        vr[r + (int64_t)(j0 + q * G) * n] = xr[q];
        vi[r + (int64_t)(j0 + q * G) * n] = xi[q];
      }
  }
  for (; ch < f.nchild; ++ch) {
    const int rr = p.rmap[p.crmap[f.child + ch] + r];
    if (rr < 0) continue;
    const FrontDev &cf = p.F[p.cfront[f.child + ch]];
    const T *cr = p.num + cf.voff + cf.s + rr;
    const T *ci = cr + (int64_t)cf.n * mr;
    for (int j = rs.g; j < nrhs; j += G) {
      vr[r + (int64_t)j * n] += cr[(int64_t)j * cf.n];
      vi[r + (int64_t)j * n] += ci[(int64_t)j * cf.n];
    }
  }
}

// z = D^-1 y on the fully-summed rows [it.i, it.i + 256), y read from W (a
// 2 x 2 block is applied by the thread of its first row).
template <typename T>
__global__ __launch_bounds__(256) void k_ffin(KP<T> p, int64_t first, int nrhs) {
  if (gated(p)) return;
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const RowSplit rs = row_split(min(256, f.s - it.i), 256, 256);
  const int n = f.n, a = it.i + rs.r, G = rs.G;
  if (a >= f.s) return;
  const int64_t sa = f.soff + a;
  const int pd = p.pdel[sa];
  if (pd < 0) return;
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)n * p.mr;
  const T *yr = p.num + f.woff;   // y = Z P v_s, left in W by its product
  const T *yi = yr + (int64_t)n * f.wcols;
  const cd d = p.dinv[sa];
  const cd d1 = pd ? p.dinv[sa + 1] : cd{0, 0}, od = pd ? p.doff[sa] : cd{0, 0};
  // eight of this thread's right-hand sides at a time: all loads, then the
  // stores (the second row of a 2 x 2 block is a valid row whenever pd == 1)
  for (int j0 = rs.g; j0 < nrhs; j0 += 8 * G) {
    double y0r[8], y0i[8], y1r[8], y1i[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t o = a + (int64_t)min(j0 + q * G, nrhs - 1) * n;
      y0r[q] = yr[o];
      y0i[q] = yi[o];
      y1r[q] = pd ? (double)yr[o + 1] : 0.0;
      y1i[q] = pd ? (double)yi[o + 1] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (j0 + q * G >= nrhs) break;
      const int64_t o = a + (int64_t)(j0 + q * G) * n;
      if (pd == 0) {
        vr[o] = (T)(d.re * y0r[q] - d.im * y0i[q]);
        vi[o] = (T)(d.re * y0i[q] + d.im * y0r[q]);
      } else {
        vr[o] = (T)((d.re * y0r[q] - d.im * y0i[q]) + (od.re * y1r[q] - od.im * y1i[q]));
        vi[o] = (T)((d.re * y0i[q] + d.im * y0r[q]) + (od.re * y1i[q] + od.im * y1r[q]));
        vr[o + 1] = (T)((od.re * y0r[q] - od.im * y0i[q]) + (d1.re * y1r[q] - d1.im * y1i[q]));
        vi[o + 1] = (T)((od.re * y0i[q] + od.im * y0r[q]) + (d1.re * y1i[q] + d1.im * y1r[q]));
      }
    }
  }
}

// Update rows [it.i, it.i + 256) (>= s) of the front vector from the parent
// front's vector, which the backward sweep has completed one level up (every
// row of it holds the solution: fully-summed rows solved there, update rows
// copied from its own parent); a few hundred rows per right-hand side instead
// of a gather across the global vector.
template <typename T>
__global__ __launch_bounds__(256) void k_binit(KP<T> p, int64_t first, int nrhs) {
  if (gated(p)) return;
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  if (skipped(p, f)) return;
  const RowSplit rs = row_split(min(256, f.n - it.i), 256, 256);
  const int n = f.n, r = it.i + rs.r, G = rs.G;
  if (r >= n) return;
  const int64_t mr = p.mr;
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)n * mr;
  const FrontDev &pf = p.F[f.parent];
  const int64_t ld = pf.n;
  const T *sr = p.num + pf.voff;
  const T *si = sr + ld * mr;
  const int64_t row = p.urow[f.uoff + r - f.s];
  for (int j0 = rs.g; j0 < nrhs; j0 += 8 * G) {
    T xr[8], xi[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int j = min(j0 + q * G, nrhs - 1);
      xr[q] = sr[row + (int64_t)j * ld];
      xi[q] = si[row + (int64_t)j * ld];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (j0 + q * G < nrhs) {
        vr[r + (int64_t)(j0 + q * G) * n] = xr[q];
        vi[r + (int64_t)(j0 + q * G) * n] = xi[q];
      }
  }
}

// Fully-summed rows [it.i, it.i + 256) of the front vector to the global
// solution vector.
template <typename T>
__global__ __launch_bounds__(256) void k_bfin(KP<T> p, int64_t first, int nrhs) {
  if (gated(p)) return;
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  if (skipped(p, f)) return;
  const RowSplit rs = row_split(min(256, f.s - it.i), 256, 256);
  const int n = f.n, r = it.i + rs.r, G = rs.G;
  if (r >= f.s) return;
  const int64_t mr = p.mr;
  const T *vr = p.num + f.voff;
  const T *vi = vr + (int64_t)n * mr;
  const bool aux = f.kind == FK_AUX;
  const int64_t ld = aux ? p.n_mult : p.n_torn;
  T *dr = p.num + (aux ? p.vl : p.vx);
  T *di = dr + ld * mr;
  const int64_t row = f.vbase + p.vars[f.idx + r];
  for (int j0 = rs.g; j0 < nrhs; j0 += 8 * G) {
    T xr[8], xi[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int j = min(j0 + q * G, nrhs - 1);
      xr[q] = vr[r + (int64_t)j * n];
      xi[q] = vi[r + (int64_t)j * n];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (j0 + q * G < nrhs) {
        dr[row + (int64_t)(j0 + q * G) * ld] = xr[q];
        di[row + (int64_t)(j0 + q * G) * ld] = xi[q];
      }
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
  if (gated(p)) return;
  __shared__ T sr[NB][65], si[NB][65];
  __shared__ T yr[NB][NB + 1], yi[NB][NB + 1];
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, s = f.s, tid = threadIdx.x;
  const int64_t mr = p.mr;
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)n * mr;
  const T *fr = p.num + f.loff;   // stored factor
  const T *fi = fr + f.lpim;
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
  if (gated(p)) return;
  if (skipped(p, p.F[p.items[first + blockIdx.x].f])) return;
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
  const T *fr = p.num + f.loff;   // stored factor
  const T *fi = fr + f.lpim;
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

// Substitutions through a front whose fully-summed block carries Z = L11^-1
// (formed during the factorisation, P basis, strict lower triangle, unit
// diagonal), as split products: every item computes one 64-output tile over
// one K chunk of ZKC into its own partial slot (64 x mr, planar), and the
// reduction kernel sums a tile's slots in a fixed order (deterministic) and
// applies the epilogue.
//   M = 0: y(r) = sum_{c <= r} Z(r, c) v(P c)        r < s        -> W, v_s
//   M = 1: u(r) = sum_{c < s}  L(r, c) y(c)          s <= r < n   -> v_R -= u
//   M = 2: u(c) = sum_{s <= r < n} L(r, c) x(r)      c < s        -> W = z - u
//   M = 3: x(a) = sum_{c >= a} Z(c, a) t(c)          a < s        -> v(P a)
// Up to 8 right-hand sides: an input row is staged in LDS as 16 contiguous
// values (8 real parts, then 8 imaginary parts), the 16 real columns of the
// matrix-core products below; more: the 64-column complex MFMA tile.
//
// The 8-RHS split products on the matrix cores: per output tile two real
// products, P = Re(A) [Re x | Im x] and Q = Im(A) [Re x | Im x] (16 real
// columns, none padded), then Re y = P(:, 0:8) - Q(:, 8:16) and
// Im y = P(:, 8:16) + Q(:, 0:8).  Each of the four waves owns 16 outputs.
// Column of result element i of a 16 x 16 block (first MFMA operand from the
// right-hand sides): FP32 4 (lane / 16) + i, FP64 lane / 16 + 4 i; its row
// is lane % 16.
template <typename T>
__device__ __forceinline__ int mfma_col(int lane, int i) {
  return sizeof(T) == 8 ? (lane >> 4) + 4 * i : (lane >> 4) * 4 + i;
}
// combines P, Q through ps (4 x 2 x 16 x 17, may alias the caller's staging
// buffers: a barrier comes first) and hands output o (0..63) of right-hand
// side q < nrhs to out(o, q, re, im)
template <typename T, class OUT>
__device__ __forceinline__ void zq_combine(T *ps, const typename V4<T>::t &P, const typename V4<T>::t &Q, int nrhs,
                                           OUT out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, m = lane & 15;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = mfma_col<T>(lane, i);
    ps[((w * 2 + 0) * 16 + m) * 17 + c] = P[i];
    ps[((w * 2 + 1) * 16 + m) * 17 + c] = Q[i];
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int q = (lane >> 4) + 4 * h;
    if (q < nrhs) {
      const T *pp = ps + (w * 2 * 16 + m) * 17, *qq = ps + ((w * 2 + 1) * 16 + m) * 17;
      out(16 * w + m, q, pp[q] - qq[8 + q], pp[8 + q] + qq[q]);
    }
  }
}
// The epilogue of a split product for output o (row it.i + o) and right-hand
// side q, given its complete sum (re, im):
//   M = 0: W = y (the diagonal-block pass reads y there)
//   M = 1: v_R -= u
//   M = 2: W = z - u
//   M = 3: v(P a) = x
template <typename T, int M>
__device__ __forceinline__ void zq_final(const KP<T> &p, const FrontDev &f, int i0, int o, int q, T re, T im) {
  const int n = f.n, x = i0 + o;
  if (x >= (M == 1 ? n : f.s)) return;
  T *vr = p.num + f.voff;
  T *vi = vr + (int64_t)n * p.mr;
  T *Wr = p.num + f.woff;
  T *Wi = Wr + (int64_t)n * f.wcols;
  const int64_t v = x + (int64_t)q * n;
  if (M == 0) {
    Wr[v] = re;
    Wi[v] = im;
  } else if (M == 1) {
    // a front without children has no extend-add sums in its update rows
    // (the gather left them alone): 0 - u, as if a zero had been stored
    const T br = f.nchild ? vr[v] : T(0), bi = f.nchild ? vi[v] : T(0);
    vr[v] = br - re;
    vi[v] = bi - im;
  } else if (M == 2) {
    Wr[v] = vr[v] - re;
    Wi[v] = vi[v] - im;
  } else {
    const int64_t d = (x / NB) * NB + p.perm[f.soff + x] + (int64_t)q * n;
    vr[d] = re;
    vi[d] = im;
  }
}
// an item whose output tile has one K chunk (it.k < 0) applies the epilogue
// itself; the others write their partial slot
template <typename T, int M>
__device__ __forceinline__ void zq_result(const KP<T> &p, const FrontDev &f, const Item &it, T *ps,
                                          const typename V4<T>::t &P, const typename V4<T>::t &Q, int nrhs) {
  if (it.k < 0) {
    zq_combine<T>(ps, P, Q, nrhs, [&](int o, int q, T re, T im) { zq_final<T, M>(p, f, it.i, o, q, re, im); });
  } else {
    const int64_t mr = p.mr;
    T *slot = p.num + p.part + (int64_t)it.k * 128 * mr;
    zq_combine<T>(ps, P, Q, nrhs, [&](int o, int q, T re, T im) {
      slot[(int64_t)q * 64 + o] = re;
      slot[64 * mr + (int64_t)q * 64 + o] = im;
    });
  }
}

// M = 0, 1 (A(o, k) a row block of the front, contiguous along o)
template <typename T, int M>
__global__ __launch_bounds__(256) void k_zq_n(KP<T> p, int64_t first, int nrhs) {
  if (gated(p)) return;
  __shared__ __align__(16) T xs[ZKC * 16];
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, s = f.s, i0 = it.i, c0 = it.j, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int cend = min(c0 + ZKC, M == 0 ? min(s, i0 + 64) : s);
  const int rlim = M == 0 ? s : n;
  const int64_t mr = p.mr;
  const T *fr = p.num + f.loff;   // stored factor
  const T *fi = fr + f.lpim;
  const T *inr = M == 0 ? p.num + f.voff : p.num + f.woff;
  const T *ini = inr + (int64_t)n * (M == 0 ? mr : f.wcols);
  const int32_t *pm = p.perm + f.soff;
  for (int e = tid; e < ZKC * 8; e += 256) {
    const int c = e % ZKC, q = e / ZKC, cc = c0 + c;
    T br = 0, bi = 0;
    if (cc < cend && q < nrhs) {
      const int src = M == 0 ? (cc / NB) * NB + pm[cc] : cc;
      const int64_t io = src + (int64_t)q * n;
      br = inr[io];
      bi = ini[io];
    }
    xs[c * 16 + q] = br;
    xs[c * 16 + 8 + q] = bi;
  }
  __syncthreads();
  const int m = lane & 15, kq = lane >> 4, r = i0 + 16 * w + m;
  const bool live = r < rlim;
  const int rc = min(r, rlim - 1);
  typename V4<T>::t P = {0, 0, 0, 0}, Q = {0, 0, 0, 0};
  // 32 columns per iteration: all loads first (clamped columns, masked
  // afterwards; the staged right-hand sides are zero past cend)
  for (int kb = c0; kb < cend; kb += 32) {
    T ar[8], ai[8], bv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = kb + 4 * u + kq;
      const int64_t e = rc + (int64_t)min(c, cend - 1) * n;
      ar[u] = fr[e];
      ai[u] = fi[e];
      bv[u] = xs[(kb - c0 + 4 * u + kq) * 16 + m];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = kb + 4 * u + kq;
      T xr = ar[u], xi = ai[u];
      if (M == 0 && c >= r) {
        xr = c == r ? T(1) : T(0);
        xi = 0;
      }
      const bool in = live && c < cend;
      P = mfma16(bv[u], in ? xr : T(0), P);
      Q = mfma16(bv[u], in ? xi : T(0), Q);
    }
  }
  zq_result<T, M>(p, f, it, xs, P, Q, nrhs);
}

// M = 2, 3 (A(o, k) a column block read along its rows k): 64 x 64 tiles of
// the front staged in LDS with coalesced loads
template <typename T, int M>
__global__ __launch_bounds__(256) void k_zq_t(KP<T> p, int64_t first, int nrhs) {
  if (gated(p)) return;
  __shared__ T at[2][64][65];
  __shared__ __align__(16) T xs[64 * 16];
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  if (skipped(p, f)) return;
  const int n = f.n, s = f.s, i0 = it.i, k0 = it.j, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int kend = min(k0 + ZKC, M == 2 ? n : s);
  const int64_t mr = p.mr;
  const T *fr = p.num + f.loff;   // stored factor
  const T *fi = fr + f.lpim;
  const T *inr = M == 2 ? p.num + f.voff : p.num + f.woff;
  const T *ini = inr + (int64_t)n * (M == 2 ? mr : f.wcols);
  const int m = lane & 15, kq = lane >> 4;
  typename V4<T>::t P = {0, 0, 0, 0}, Q = {0, 0, 0, 0};
  for (int rb = k0; rb < kend; rb += 64) {
    __syncthreads();
    T tv[2][16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + 256 * u, rr = e & 63, cc = e >> 6;
      const int row = min(rb + rr, kend - 1), col = min(i0 + cc, s - 1);
      const int64_t x = row + (int64_t)col * n;
      tv[0][u] = fr[x];
      tv[1][u] = fi[x];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + 256 * u, rr = e & 63, cc = e >> 6, row = rb + rr, col = i0 + cc;
      T vr = tv[0][u], vi = tv[1][u];
      if (row >= kend || col >= s || (M == 3 && row <= col)) {
        vr = (M == 3 && row == col && row < kend && col < s) ? T(1) : T(0);
        vi = 0;
      }
      at[0][rr][cc] = vr;
      at[1][rr][cc] = vi;
    }
    for (int e = tid; e < 64 * 8; e += 256) {
      const int rr = e & 63, q = e >> 6, row = rb + rr;
      T br = 0, bi = 0;
      if (row < kend && q < nrhs) {
        const int64_t x = row + (int64_t)q * n;
        br = inr[x];
        bi = ini[x];
      }
      xs[rr * 16 + q] = br;
      xs[rr * 16 + 8 + q] = bi;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 64; kk += 4) {
      const T ar = at[0][kk + kq][16 * w + m], ai = at[1][kk + kq][16 * w + m];
      const T b = xs[(kk + kq) * 16 + m];
      P = mfma16(b, ar, P);
      Q = mfma16(b, ai, Q);
    }
  }
  zq_result<T, M>(p, f, it, &at[0][0][0], P, Q, nrhs);
}

// The same split products on the MFMA GEMM tile, for many right-hand sides
// (64 at a time): the vector-unit kernels above re-read the front once per 8
// columns.
template <typename T, int M>
__device__ __forceinline__ void zslot_out(const KP<T> &p, const FrontDev &f, const Item &it,
                                          const typename V4<T>::t (&cr)[2][2], const typename V4<T>::t (&ci)[2][2],
                                          int j0, int nrhs) {
  const int64_t mr = p.mr;
  T *slot = p.num + p.part + (int64_t)max(it.k, 0) * 128 * mr;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int o = out_row(x), j = j0 + out_col<T>(y, i);
        if (j < nrhs) {
          if (it.k < 0) {
            zq_final<T, M>(p, f, it.i, o, j, cr[x][y][i], ci[x][y][i]);
          } else {
            slot[(int64_t)j * 64 + o] = cr[x][y][i];
            slot[64 * mr + (int64_t)j * 64 + o] = ci[x][y][i];
          }
        }
      }
}

// M = 0, 1: A(o, k) is a row block of the front (contiguous along o)
// three waves per SIMD (no spills at that register budget)
template <typename T, int M>
__global__ __launch_bounds__(256, 3) void k_zmma_n(KP<T> p, int64_t first, int nrhs) {
  if (gated(p)) return;
  __shared__ GemmSmem<T, T64> sm;
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int n = f.n, s = f.s, i0 = it.i, c0 = it.j;
  const int cend = min(c0 + ZKC, M == 0 ? min(s, i0 + 64) : s);
  const int rlim = M == 0 ? s : n;
  const int64_t mr = p.mr;
  const T *fr = p.num + f.loff;   // stored factor
  const T *fi = fr + f.lpim;
  const T *inr = M == 0 ? p.num + f.voff : p.num + f.woff;
  const T *ini = inr + (int64_t)n * (M == 0 ? mr : f.wcols);
  const int32_t *pm = p.perm + f.soff;
  auto fa = [&](int m, int kk, T &re, T &im) {
    const int r = i0 + m;
    if (r < rlim) {
      if (M != 0 || kk < r) {
        const int64_t e = r + (int64_t)kk * n;
        re = fr[e];
        im = fi[e];
      } else if (kk == r) {
        re = 1;
      }
    }
  };
  for (int j0 = 0; j0 < nrhs; j0 += 64) {
    auto fb = [&](int c, int kk, T &re, T &im) {
      if (j0 + c < nrhs) {
        const int src = M == 0 ? (kk / NB) * NB + pm[kk] : kk;
        const int64_t e = src + (int64_t)(j0 + c) * n;
        re = inr[e];
        im = ini[e];
      }
    };
    typename V4<T>::t cr[2][2], ci[2][2];
    gemm_tile<T, T64, false, true>(sm, c0, cend, fa, fb, cr, ci);
    zslot_out<T, M>(p, f, it, cr, ci, j0, nrhs);
  }
}

// M = 2, 3: A(o, k) is a column block of the front read along its rows k
template <typename T, int M>
__global__ __launch_bounds__(256) void k_zmma_t(KP<T> p, int64_t first, int nrhs) {
  if (gated(p)) return;
  __shared__ GemmSmem<T, T64> sm;
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  if (skipped(p, f)) return;
  const int n = f.n, s = f.s, i0 = it.i, k0 = it.j;
  const int kend = min(k0 + ZKC, M == 2 ? n : s);
  const int64_t mr = p.mr;
  const T *fr = p.num + f.loff;   // stored factor
  const T *fi = fr + f.lpim;
  const T *inr = M == 2 ? p.num + f.voff : p.num + f.woff;
  const T *ini = inr + (int64_t)n * (M == 2 ? mr : f.wcols);
  auto fa = [&](int m, int kk, T &re, T &im) {
    const int col = i0 + m;
    if (col < s) {
      if (M == 2 || kk > col) {
        const int64_t e = kk + (int64_t)col * n;
        re = fr[e];
        im = fi[e];
      } else if (kk == col) {
        re = 1;
      }
    }
  };
  for (int j0 = 0; j0 < nrhs; j0 += 64) {
    auto fb = [&](int c, int kk, T &re, T &im) {
      if (j0 + c < nrhs) {
        const int64_t e = kk + (int64_t)(j0 + c) * n;
        re = inr[e];
        im = ini[e];
      }
    };
    typename V4<T>::t cr[2][2], ci[2][2];
    gemm_tile<T, T64, true, true>(sm, k0, kend, fa, fb, cr, ci);
    zslot_out<T, M>(p, f, it, cr, ci, j0, nrhs);
  }
}

// Reduction of the partial slots [it.k, it.k + it.j) of output tile it.i
// (fixed order: deterministic), then the product's epilogue.
template <typename T, int M>
__global__ __launch_bounds__(256) void k_zred(KP<T> p, int64_t first, int nrhs) {
  if (gated(p)) return;
  const Item it = p.items[first + blockIdx.x];
  const FrontDev f = p.F[it.f];
  if (M >= 2 && skipped(p, f)) return;   // backward reductions only
  const int64_t mr = p.mr;
  const T *part = p.num + p.part;
  const int hi = M == 1 ? f.n : f.s;
  // rows of the tile times columns, R = 8 ... 64 rows per column
  const RowSplit rs = row_split(min(64, hi - it.i), 64, 256);
  const int R = 1 << rs.sh;
  for (int e = threadIdx.x; e < R * nrhs; e += 256) {
    const int o = e & (R - 1), j = e >> rs.sh;
    if (it.i + o >= hi) continue;
    T sr = 0, si = 0;
    for (int k = it.k; k < it.k + it.j; ++k) {
      const T *sl = part + (int64_t)k * 128 * mr + (int64_t)j * 64 + o;
      sr += sl[0];
      si += sl[64 * mr];
    }
    zq_final<T, M>(p, f, it.i, o, j, sr, si);
  }
}

// interface product on the matrix cores, for more than ZMMA_MIN right-hand
// sides: mode 0: YG = X v_root; mode 1: v_root = YG - X h; one 64-row block of X times 64-column
// blocks of the right-hand sides over the full inner dimension g
template <typename T>
__global__ __launch_bounds__(256) void k_xmma(KP<T> p, int mode, int nrhs) {
  if (gated(p)) return;
  if (mode == 1 && skipped(p, p.F[p.gemv[blockIdx.x].f])) return;
  __shared__ GemmSmem<T, T64> sm;
  const Item it = p.gemv[blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int g = f.s, i0 = it.i;
  const int64_t mr = p.mr, pl = (int64_t)g * mr;
  const T *Xr = p.num + f.xoff;
  const T *Xi = Xr + (int64_t)g * g;
  T *yg = p.num + f.goff;
  T *v = p.num + f.voff;
  const T *in = mode == 0 ? v : yg + 2 * pl;
  auto fa = [&](int m, int kk, T &re, T &im) {
    const int r = i0 + m;
    if (r < g) {
      const int64_t e = r + (int64_t)kk * g;
      re = Xr[e];
      im = Xi[e];
    }
  };
  for (int j0 = 0; j0 < nrhs; j0 += 64) {
    auto fb = [&](int c, int kk, T &re, T &im) {
      if (j0 + c < nrhs) {
        const int64_t e = kk + (int64_t)(j0 + c) * g;
        re = in[e];
        im = in[e + pl];
      }
    };
    typename V4<T>::t cr[2][2], ci[2][2];
    gemm_tile<T, T64, false, true>(sm, 0, g, fa, fb, cr, ci);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = i0 + out_row(x), j = j0 + out_col<T>(y, i);
          if (r < g && j < nrhs) {
            const int64_t o = r + (int64_t)j * g;
            if (mode == 0) {
              yg[o] = cr[x][y][i];
              yg[o + pl] = ci[x][y][i];
            } else {
              v[o] = yg[o] - cr[x][y][i];
              v[o + pl] = yg[o + pl] - ci[x][y][i];
            }
          }
        }
  }
}

// interface product on the matrix cores for up to 8 right-hand sides (the
// same two modes as k_xmma): P = Re(X) [Re in | Im in], Q = Im(X) [Re in |
// Im in] over the full inner dimension g, the right-hand sides staged in LDS
// 256 columns of X at a time
template <typename T>
__global__ __launch_bounds__(256) void k_xq(KP<T> p, int mode, int nrhs) {
  if (gated(p)) return;
  if (mode == 1 && skipped(p, p.F[p.gemv[blockIdx.x].f])) return;
  __shared__ __align__(16) T xs[256 * 16];
  const Item it = p.gemv[blockIdx.x];
  const FrontDev f = p.F[it.f];
  const int g = f.s, i0 = it.i, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t mr = p.mr, pl = (int64_t)g * mr;
  const T *Xr = p.num + f.xoff;
  const T *Xi = Xr + (int64_t)g * g;
  T *yg = p.num + f.goff;
  T *v = p.num + f.voff;
  const T *in = mode == 0 ? v : yg + 2 * pl;
  const int m = lane & 15, kq = lane >> 4, r = i0 + 16 * w + m;
  const bool live = r < g;
  const int rc = min(r, g - 1);
  typename V4<T>::t P = {0, 0, 0, 0}, Q = {0, 0, 0, 0};
  for (int c0 = 0; c0 < g; c0 += 256) {
    const int cend = min(c0 + 256, g);
    __syncthreads();
    for (int e = tid; e < 256 * 8; e += 256) {
      const int c = e % 256, q = e / 256, cc = c0 + c;
      T br = 0, bi = 0;
      if (cc < cend && q < nrhs) {
        const int64_t io = cc + (int64_t)q * g;
        br = in[io];
        bi = in[io + pl];
      }
      xs[c * 16 + q] = br;
      xs[c * 16 + 8 + q] = bi;
    }
    __syncthreads();
    for (int kb = c0; kb < cend; kb += 32) {
      T ar[8], ai[8], bv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = kb + 4 * u + kq;
        const int64_t e = rc + (int64_t)min(c, cend - 1) * g;
        ar[u] = Xr[e];
        ai[u] = Xi[e];
        bv[u] = xs[(kb - c0 + 4 * u + kq) * 16 + m];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool ok = live && kb + 4 * u + kq < cend;
        P = mfma16(bv[u], ok ? ar[u] : T(0), P);
        Q = mfma16(bv[u], ok ? ai[u] : T(0), Q);
      }
    }
  }
  zq_combine<T>(xs, P, Q, nrhs, [&](int o, int q, T re, T im) {
    const int row = i0 + o;
    if (row >= g) return;
    const int64_t x = row + (int64_t)q * g;
    if (mode == 0) {
      yg[x] = re;
      yg[x + pl] = im;
    } else {
      v[x] = yg[x] - re;
      v[x + pl] = yg[x + pl] - im;
    }
  });
}

// d(p) = sum_t s_t YG_t - c(p)
template <typename T>
__global__ __launch_bounds__(256) void k_mgather(KP<T> p, int nrhs, int with_c) {
  if (gated(p)) return;
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
  if (gated(p)) return;
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
  if (!which && p.dmask) {
    // domain of torn row r (rows are contiguous per domain)
    int lo = 0, hi = p.n_dom;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (p.domrow[mid] <= r) lo = mid;
      else hi = mid;
    }
    if (!p.dmask[lo]) return;
  }
  const T *s = p.num + (which ? p.vl : p.vx);
  u[r + j * ldu] = cd{(double)s[r + j * rows], (double)s[r + j * rows + rows * p.mr]};
}

// Selected rows of the internal solution: out(i, j) = x(rows[i], j).
template <typename T>
__global__ void k_sel_out(KP<T> p, const int64_t *rows, int64_t nsel, cd *out, int64_t ldo, int nrhs) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nsel * nrhs) return;
  const int64_t i = e % nsel, j = e / nsel, r = rows[i];
  const T *s = p.num + p.vx;
  out[i + j * ldo] = cd{(double)s[r + j * p.n_torn], (double)s[r + j * p.n_torn + p.n_torn * p.mr]};
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

// FP64 refinement state: U, torn rows x mr columns with a row's columns
// contiguous (complex interleaved: the residual's gathers of a row read one
// run of the columns), and L, multipliers x mr planar column-major.
// U from / plus the internal column-major planar solution x: 64-row x
// 8-column tiles through LDS, coalesced on both sides (mode 0: U = x, 1: U += x).
template <typename T>
__global__ __launch_bounds__(256) void k_r_utile(KP<T> p, int nrhs, int mode) {
  if (mode && gated(p)) return;
  __shared__ double sr[64][9], si[64][9];
  const int64_t nt = p.n_torn, mr = p.mr;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int j0 = blockIdx.y * 8;
  const T *x = p.num + p.vx;
  for (int e = threadIdx.x; e < 512; e += 256) {
    const int j = e >> 6, rr = e & 63;
    const int64_t r = r0 + rr;
    double a = 0, b = 0;
    if (r < nt && j0 + j < nrhs) {
      a = (double)x[r + (int64_t)(j0 + j) * nt];
      b = (double)x[r + (int64_t)(j0 + j) * nt + nt * mr];
    }
    sr[rr][j] = a;
    si[rr][j] = b;
  }
  __syncthreads();
  cd *U = (cd *)p.r64;
  for (int e = threadIdx.x; e < 512; e += 256) {
    const int rr = e >> 3, j = e & 7;
    const int64_t r = r0 + rr;
    if (r < nt && j0 + j < nrhs) {
      cd &u = U[r * mr + j0 + j];
      if (mode) {
        u.re += sr[rr][j];
        u.im += si[rr][j];
      } else {
        u = cd{sr[rr][j], si[rr][j]};
      }
    }
  }
}

// L from / plus the internal multipliers (mode 0: L = l, 1: L += l)
template <typename T>
__global__ void k_r_lpart(KP<T> p, int nrhs, int mode) {
  if (mode && gated(p)) return;
  const int64_t mr = p.mr;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= p.n_mult * nrhs) return;
  double *L = p.r64 + 2 * p.n_torn * mr;
  const int64_t m = e % p.n_mult, j = e / p.n_mult;
  const T *l = p.num + p.vl;
  const double a = (double)l[m + j * p.n_mult], b = (double)l[m + j * p.n_mult + p.n_mult * mr];
  if (mode) {
    L[m + j * p.n_mult] += a;
    L[m + j * p.n_mult + p.n_mult * mr] += b;
  } else {
    L[m + j * p.n_mult] = a;
    L[m + j * p.n_mult + p.n_mult * mr] = b;
  }
}

// FP64 operator copy in SELL-64 order (padding entries zero); one wave per slice
__global__ __launch_bounds__(256) void k_sell_fill(const int64_t *csrp, const int64_t *sellp, int64_t n_torn,
                                                   const cd *vals, cd *sell) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t sl = r >> 6;
  if (sl * 64 >= n_torn) return;
  const int64_t zb = sellp[sl], zw = sellp[sl + 1];
  const int64_t rb = r < n_torn ? csrp[r] : 0, len = r < n_torn ? csrp[r + 1] - rb : 0;
  int64_t k = 0;
  for (int64_t z = zb + (r & 63); z < zw; z += 64, ++k) sell[z] = k < len ? vals[rb + k] : cd{0, 0};
}

// r_u = f - K u - B^T lam ; r_l = -B u ; writes the FP32 correction rhs (vf, vc)
// and per-block sums of |r|^2 (or |f|^2 when fnorm) per column.  Columns are
// processed 8 at a time so the operator is streamed once per 8 columns.
template <typename T>
__global__ __launch_bounds__(256) void k_r_resid(KP<T> p, const cd *f, int64_t ldf, int nrhs, int64_t part_off,
                                                 int fnorm) {
  if (gated(p)) return;
  __shared__ double red[8][256];
  const int64_t mr = p.mr;
  const cd *Uc = (const cd *)p.r64;
  const double *L = p.r64 + 2 * p.n_torn * mr;
  double *part = p.r64 + part_off;
  const int64_t nrow = p.n_torn + p.n_mult;
  const int64_t nt = p.n_torn, nm = p.n_mult;
  for (int j0 = 0; j0 < nrhs; j0 += 8) {
    const int nj = min(8, nrhs - j0);
    // column offsets of the pass; columns past nrhs repeat the last one (their
    // loads are unconditional, their results are dropped)
    int64_t jc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) jc[q] = min(j0 + q, nrhs - 1);
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nrow; e += (int64_t)gridDim.x * 256) {
      double rr[8], ri[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) rr[q] = ri[q] = 0;
      if (e < nt) {
        // gr, gi: the same row of f - K u~, u~ taking every DoF's value from
        // its representative copy; summed over the copies of a DoF this is
        // the residual of the assembled (undecomposed) system
        // (gr, gi: the correction -K (u~ - u), nonzero only through columns
        // whose representative is another copy, i.e. interface DoFs)
        double gr[8], gi[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const cd fv = f[e + jc[q] * ldf];
          rr[q] = fv.re;
          ri[q] = fv.im;
          gr[q] = gi[q] = 0;
        }
        if (!fnorm) {
          // SELL-64: the wave's 64 rows form one slice, entry k of all its
          // rows is one contiguous 1 KiB run
          const int64_t zb = p.sellp[e >> 6], zw = p.sellp[(e >> 6) + 1];
#pragma unroll 2
          for (int64_t z = zb + (e & 63); z < zw; z += 64) {
            const cd a = p.vals[z];
            const int64_t c = p.sellc[z];
            const int64_t cg = p.grep[c];
            // the pass's columns of row c: one contiguous run
            const cd *uc = Uc + c * mr;
            double ur[8], ui[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const cd x = uc[jc[q]];
              ur[q] = x.re;
              ui[q] = x.im;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              rr[q] -= a.re * ur[q] - a.im * ui[q];
              ri[q] -= a.re * ui[q] + a.im * ur[q];
            }
            if (cg != c) {
              const cd *ug = Uc + cg * mr;
#pragma unroll
              for (int q = 0; q < 8; ++q) {
                const cd y = ug[jc[q]];
                const double dr = y.re - ur[q], di = y.im - ui[q];
                gr[q] -= a.re * dr - a.im * di;
                gi[q] -= a.re * di + a.im * dr;
              }
            }
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            gr[q] += rr[q];
            gi[q] += ri[q];
          }
          const int gidx = p.rowgam[e];
          if (gidx >= 0) {
            const GamRef G = p.grefs[gidx];
            for (int t = 0; t < G.cnt; ++t) {
              const int64_t m = p.hmult[G.beg + t];
              const double sg = p.hsign[G.beg + t];
#pragma unroll
              for (int q = 0; q < 8; ++q) {
                rr[q] -= sg * L[m + jc[q] * nm];
                ri[q] -= sg * L[m + jc[q] * nm + nm * mr];
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
        if (fnorm) {   // the right-hand side itself
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            gr[q] = rr[q];
            gi[q] = ri[q];
          }
        }
        double *G = p.r64 + p.rg;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (q < nj) {
            G[e + (j0 + q) * nt] = gr[q];
            G[e + (j0 + q) * nt + nt * mr] = gi[q];
          }
      } else if (!fnorm) {
        const int64_t m = e - nt;
        const MultRef R = p.mrefs[m];
        T *vc = p.num + p.vc;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            const double sg = R.sg[t];
            const cd x = Uc[R.row[t] * mr + jc[q]];
            rr[q] -= sg * x.re;
            ri[q] -= sg * x.im;
          }
          if (q < nj) {
            vc[m + (j0 + q) * nm] = (T)rr[q];
            vc[m + (j0 + q) * nm + nm * mr] = (T)ri[q];
          }
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

// Assembled residual: per global DoF (component of copies) the sum of its
// rows of f - K u~, squared and summed per column into per-block partials.
template <typename T>
__global__ __launch_bounds__(256) void k_r_gsum(KP<T> p, int nrhs, int64_t part_off) {
  if (gated(p)) return;
  __shared__ double red[8][256];
  const int64_t mr = p.mr, nt = p.n_torn;
  const double *G = p.r64 + p.rg;
  double *part = p.r64 + part_off;
  for (int j0 = 0; j0 < nrhs; j0 += 8) {
    const int nj = min(8, nrhs - j0);
    int64_t jc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) jc[q] = min(j0 + q, nrhs - 1);
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0;
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < p.n_gcomp; c += (int64_t)gridDim.x * 256) {
      double sr[8], si[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) sr[q] = si[q] = 0;
      for (int k = p.gcp[c]; k < p.gcp[c + 1]; ++k) {
        const int64_t r = p.gcr[k];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          sr[q] += G[r + jc[q] * nt];
          si[q] += G[r + jc[q] * nt + nt * mr];
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] += sr[q] * sr[q] + si[q] * si[q];
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

__global__ void k_r_reduce(const double *part, int nblk, int nrhs, double *out, const int *skip) {
  const int j = blockIdx.x;
  if (j >= nrhs || (skip && *(volatile const int *)skip)) return;
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

// Convergence test of the refinement (one workgroup).  Per column the torn
// and the assembled squared residual norms relative to the right-hand
// side's; ctl[0] is set when every column has both within tol (or a value is
// not finite: ctl[2]), ctl[1] counts the correction iterations that ran
// (count = 1 after a correction), rel receives the two maxima.  A test of an
// iteration that was skipped (ctl[0] already set) does nothing.
__global__ __launch_bounds__(256) void k_r_test(const double *norm, const double *fnorm, int nrhs, int mr, double tol,
                                                int *ctl, double *rel, int count) {
  if (*(volatile int *)ctl) return;
  __shared__ double mt[256], mg[256];
  __shared__ int bad[256];
  double rt = 0, rg = 0;
  int b = 0;
  for (int j = threadIdx.x; j < nrhs; j += 256) {
    const double t = fnorm[j] > 0 ? sqrt(norm[j] / fnorm[j]) : sqrt(norm[j]);
    const double g = fnorm[mr + j] > 0 ? sqrt(norm[mr + j] / fnorm[mr + j]) : sqrt(norm[mr + j]);
    if (!isfinite(t) || !isfinite(g)) b = 1;
    rt = fmax(rt, t);
    rg = fmax(rg, g);
  }
  mt[threadIdx.x] = rt;
  mg[threadIdx.x] = rg;
  bad[threadIdx.x] = b;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      mt[threadIdx.x] = fmax(mt[threadIdx.x], mt[threadIdx.x + st]);
      mg[threadIdx.x] = fmax(mg[threadIdx.x], mg[threadIdx.x + st]);
      bad[threadIdx.x] |= bad[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    ctl[1] += count;
    rel[0] = mt[0];
    rel[1] = mg[0];
    if (bad[0]) ctl[2] = 1;
    if (bad[0] || fmax(mt[0], mg[0]) <= tol) ctl[0] = 1;
  }
}

__global__ void k_r_ctl_reset(int *ctl) {
  if (threadIdx.x < 4) ctl[threadIdx.x] = 0;
}

// U -> the caller's u (column-major, leading dimension ldu): 64-row x
// 8-column tiles through LDS
template <typename T>
__global__ __launch_bounds__(256) void k_r_uout(KP<T> p, cd *u, int64_t ldu, int nrhs) {
  __shared__ double sr[64][9], si[64][9];
  const int64_t nt = p.n_torn, mr = p.mr;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int j0 = blockIdx.y * 8;
  const cd *U = (const cd *)p.r64;
  for (int e = threadIdx.x; e < 512; e += 256) {
    const int rr = e >> 3, j = e & 7;
    const int64_t r = r0 + rr;
    cd x = cd{0, 0};
    if (r < nt && j0 + j < nrhs) x = U[r * mr + j0 + j];
    sr[rr][j] = x.re;
    si[rr][j] = x.im;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 512; e += 256) {
    const int j = e >> 6, rr = e & 63;
    const int64_t r = r0 + rr;
    if (r < nt && j0 + j < nrhs) u[r + (int64_t)(j0 + j) * ldu] = cd{sr[rr][j], si[rr][j]};
  }
}

template <typename T>
__global__ void k_r_lout(KP<T> p, cd *lam, int64_t ldl, int nrhs) {
  const int64_t mr = p.mr;
  const double *L = p.r64 + 2 * p.n_torn * mr;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= p.n_mult * nrhs) return;
  const int64_t m = e % p.n_mult, j = e / p.n_mult;
  lam[m + j * ldl] = cd{L[m + j * p.n_mult], L[m + j * p.n_mult + p.n_mult * mr]};
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
  k.urow = (const int32_t *)(m + P.m_urow);
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
  k.sellp = (const int64_t *)(m + P.m_sellp);
  k.sellc = (const int32_t *)(m + P.m_sellc);
  k.domrow = (const int64_t *)(m + P.m_domrow);
  k.dmask = nullptr;
  k.gemv = (const Item *)(m + P.m_gemv);
  k.grep = (const int32_t *)(m + P.m_grep);
  k.gcp = (const int32_t *)(m + P.m_gcp);
  k.gcr = (const int32_t *)(m + P.m_gcr);
  k.n_gcomp = P.n_gcomp;
  k.rg = P.r_g;
  k.skip = nullptr;
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
  k.n_dom = P.n_dom;
  return k;
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename T>
static hipError_t run_seq(const Plan &P, const KP<T> &k, const std::vector<Launch> &seq, int nrhs, hipStream_t main,
                          KTimer *tm, const SideStream *side = nullptr) {
  const bool two = side && side->stream[0] && side->stream[1];
  for (const Launch &L : seq) {
    if (L.kind == L_FORK || L.kind == L_JOIN) {
      if (!two) continue;
      const int x = L.side - 1;
      hipEvent_t e = (hipEvent_t)(L.kind == L_FORK ? side->fork[x] : side->join[x]);
      hipStream_t from = L.kind == L_FORK ? main : (hipStream_t)side->stream[x];
      hipStream_t to = L.kind == L_FORK ? (hipStream_t)side->stream[x] : main;
      hipError_t r = hipEventRecord(e, from);
      if (r == hipSuccess) r = hipStreamWaitEvent(to, e, 0);
      if (r != hipSuccess) return r;
      continue;
    }
    hipStream_t st = two && L.side ? (hipStream_t)side->stream[L.side - 1] : main;
    dim3 g(L.count), b(256);
    const bool timed = tm && tm->kind == (L.kind == L_SYRK2 ? (int)L_SYRK : L.kind) && tm->used + 2 <= tm->cap;
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
      case L_PANEL: hipLaunchKernelGGL(k_panel<T>, g, dim3(256), 0, st, k, L.first); break;
      case L_TRSM: hipLaunchKernelGGL(k_trsm<T>, g, b, 0, st, k, L.first); break;
      case L_SYRK: hipLaunchKernelGGL((k_syrk<T, T64>), g, b, 0, st, k, L.first); break;
      case L_SYRK2: hipLaunchKernelGGL((k_syrk<T, T128>), g, dim3(T128::NTH), 0, st, k, L.first); break;
      case L_UPDPANEL: hipLaunchKernelGGL(k_updpanel<T>, g, b, 0, st, k, L.first); break;
      case L_ZREC1: hipLaunchKernelGGL(k_zrec1<T>, g, b, 0, st, k, L.first); break;
      case L_ZREC2: hipLaunchKernelGGL(k_zrec2<T>, g, b, 0, st, k, L.first); break;
      case L_DINVZ: hipLaunchKernelGGL(k_dinvz<T>, g, b, 0, st, k, L.first); break;
      case L_STORE: hipLaunchKernelGGL(k_store<T>, g, b, 0, st, k, L.first); break;
      case L_INVSYRK: hipLaunchKernelGGL(k_invsyrk<T>, g, b, 0, st, k, L.first); break;
      case S_FINIT: hipLaunchKernelGGL(k_finit<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_FFIN: hipLaunchKernelGGL(k_ffin<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_BINIT: hipLaunchKernelGGL(k_binit<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_BFIN: hipLaunchKernelGGL(k_bfin<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_FFRONT: hipLaunchKernelGGL(k_ffront<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_BFRONT: hipLaunchKernelGGL(k_bfront<T>, g, b, 0, st, k, L.first, nrhs); break;
      case S_ZP0:
        if (nrhs > ZMMA_MIN) hipLaunchKernelGGL((k_zmma_n<T, 0>), g, b, 0, st, k, L.first, nrhs);
        else hipLaunchKernelGGL((k_zq_n<T, 0>), g, b, 0, st, k, L.first, nrhs);
        break;
      case S_ZR0: hipLaunchKernelGGL((k_zred<T, 0>), g, b, 0, st, k, L.first, nrhs); break;
      case S_ZP1:
        if (nrhs > ZMMA_MIN) hipLaunchKernelGGL((k_zmma_n<T, 1>), g, b, 0, st, k, L.first, nrhs);
        else hipLaunchKernelGGL((k_zq_n<T, 1>), g, b, 0, st, k, L.first, nrhs);
        break;
      case S_ZR1: hipLaunchKernelGGL((k_zred<T, 1>), g, b, 0, st, k, L.first, nrhs); break;
      case S_ZP2:
        if (nrhs > ZMMA_MIN) hipLaunchKernelGGL((k_zmma_t<T, 2>), g, b, 0, st, k, L.first, nrhs);
        else hipLaunchKernelGGL((k_zq_t<T, 2>), g, b, 0, st, k, L.first, nrhs);
        break;
      case S_ZR2: hipLaunchKernelGGL((k_zred<T, 2>), g, b, 0, st, k, L.first, nrhs); break;
      case S_ZP3:
        if (nrhs > ZMMA_MIN) hipLaunchKernelGGL((k_zmma_t<T, 3>), g, b, 0, st, k, L.first, nrhs);
        else hipLaunchKernelGGL((k_zq_t<T, 3>), g, b, 0, st, k, L.first, nrhs);
        break;
      case S_ZR3: hipLaunchKernelGGL((k_zred<T, 3>), g, b, 0, st, k, L.first, nrhs); break;
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
  if (threadIdx.x < 5) status[threadIdx.x] = threadIdx.x == 4 ? 0x7fffffff : 0;
}

template <typename T>
static hipError_t factor_t(const Plan &P, uint8_t *ws, const void *vals, hipStream_t st, KTimer *tm,
                           const SideStream *side) {
  KP<T> k = make_kp<T>(P, ws, vals);
  hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(64), 0, st, k.status);
  return run_seq<T>(P, k, P.factor_seq, 0, st, tm, side);
}

template <typename T>
static hipError_t solve_core_t(const Plan &P, uint8_t *ws, int nrhs, bool with_c, hipStream_t st, KTimer *tm,
                               bool subset, const int *gate) {
  KP<T> k = make_kp<T>(P, ws, nullptr);
  if (subset) k.dmask = ws + P.b_dmask;
  k.skip = gate;
  hipError_t e = run_seq<T>(P, k, P.solve_dom_fwd, nrhs, st, tm);
  if (e != hipSuccess) return e;
  if (!P.gemv_items.empty())
    hipLaunchKernelGGL(nrhs > ZMMA_MIN ? k_xmma<T> : k_xq<T>, dim3(P.gemv_items.size()), dim3(256), 0, st, k, 0,
                       nrhs);
  if (P.n_mult > 0)
    hipLaunchKernelGGL(k_mgather<T>, dim3(nblk(P.n_mult * nrhs)), dim3(256), 0, st, k, nrhs, with_c ? 1 : 0);
  e = run_seq<T>(P, k, P.solve_aux, nrhs, st, tm);
  if (e != hipSuccess) return e;
  if (!P.grefs.empty())
    hipLaunchKernelGGL(k_hgather<T>, dim3(nblk((int64_t)P.grefs.size() * nrhs)), dim3(256), 0, st, k,
                       (int64_t)P.grefs.size(), nrhs);
  if (!P.gemv_items.empty())
    hipLaunchKernelGGL(nrhs > ZMMA_MIN ? k_xmma<T> : k_xq<T>, dim3(P.gemv_items.size()), dim3(256), 0, st, k, 1,
                       nrhs);
  e = run_seq<T>(P, k, P.solve_dom_bwd, nrhs, st, tm);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t run_launch(const Plan &P, uint8_t *ws, const Launch &L, hipStream_t st) {
  const std::vector<Launch> seq{L};
  if (P.precision == 0) return run_seq<double>(P, make_kp<double>(P, ws, nullptr), seq, 0, st, nullptr);
  return run_seq<float>(P, make_kp<float>(P, ws, nullptr), seq, 0, st, nullptr);
}

hipError_t factor(const Plan &P, uint8_t *ws, const void *vals, hipStream_t st, KTimer *tm, const SideStream *side) {
  return P.precision == 0 ? factor_t<double>(P, ws, vals, st, tm, side) : factor_t<float>(P, ws, vals, st, tm, side);
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

hipError_t solve_core(const Plan &P, uint8_t *ws, int nrhs, bool with_c, hipStream_t st, KTimer *tm, bool subset,
                      const int *gate) {
  return P.precision == 0 ? solve_core_t<double>(P, ws, nrhs, with_c, st, tm, subset, gate)
                          : solve_core_t<float>(P, ws, nrhs, with_c, st, tm, subset, gate);
}

hipError_t sol_out(const Plan &P, uint8_t *ws, void *u, int64_t ldu, void *lam, int64_t ldl, int nrhs,
                   hipStream_t st, bool subset) {
  if (P.precision == 0) {
    KP<double> k = make_kp<double>(P, ws, nullptr);
    if (subset) k.dmask = ws + P.b_dmask;
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

hipError_t sel_out(const Plan &P, uint8_t *ws, int64_t nsel, void *out, int64_t ldo, int nrhs, hipStream_t st) {
  if (nsel == 0) return hipSuccess;
  const int64_t *rows = (const int64_t *)(ws + P.b_sel);
  if (P.precision == 0)
    hipLaunchKernelGGL(k_sel_out<double>, dim3(nblk(nsel * nrhs)), dim3(256), 0, st, make_kp<double>(P, ws, nullptr),
                       rows, nsel, (cd *)out, ldo, nrhs);
  else
    hipLaunchKernelGGL(k_sel_out<float>, dim3(nblk(nsel * nrhs)), dim3(256), 0, st, make_kp<float>(P, ws, nullptr),
                       rows, nsel, (cd *)out, ldo, nrhs);
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
hipError_t operator_copy(const Plan &P, uint8_t *ws, const void *vals, hipStream_t st) {
  if (P.n_torn == 0) return hipSuccess;
  const uint8_t *m = ws + P.b_meta;
  hipLaunchKernelGGL(k_sell_fill, dim3(nblk(((P.n_torn + 63) / 64) * 64)), dim3(256), 0, st,
                     (const int64_t *)(m + P.m_csrp), (const int64_t *)(m + P.m_sellp), P.n_torn, (const cd *)vals,
                     (cd *)(ws + P.b_vals));
  return hipGetLastError();
}
static hipError_t refine_state(const Plan &P, uint8_t *ws, int nrhs, hipStream_t st, const int *gate, int mode) {
  KP<float> k = make_kp<float>(P, ws, ws + P.b_vals);
  k.skip = gate;
  if (P.n_torn > 0)
    hipLaunchKernelGGL(k_r_utile<float>, dim3((unsigned)((P.n_torn + 63) / 64), (unsigned)((nrhs + 7) / 8)),
                       dim3(256), 0, st, k, nrhs, mode);
  if (P.n_mult > 0)
    hipLaunchKernelGGL(k_r_lpart<float>, dim3(nblk(P.n_mult * nrhs)), dim3(256), 0, st, k, nrhs, mode);
  return hipGetLastError();
}
hipError_t refine_init(const Plan &P, uint8_t *ws, int nrhs, hipStream_t st) {
  return refine_state(P, ws, nrhs, st, nullptr, 0);
}
hipError_t refine_update(const Plan &P, uint8_t *ws, int nrhs, hipStream_t st, const int *gate) {
  return refine_state(P, ws, nrhs, st, gate, 1);
}
hipError_t refine_resid(const Plan &P, uint8_t *ws, const void *f, int64_t ldf, int nrhs, bool fnorm,
                        hipStream_t st, const int *gate) {
  KP<float> k = make_kp<float>(P, ws, ws + P.b_vals);
  k.skip = gate;
  const int nb = (int)P.r_nblk;
  hipLaunchKernelGGL(k_r_resid<float>, dim3(nb), dim3(256), 0, st, k, (const cd *)f, ldf, nrhs, P.r_part,
                     fnorm ? 1 : 0);
  double *r64 = (double *)(ws + P.b_r64);
  double *out = r64 + (fnorm ? P.r_fnorm : P.r_norm);
  hipLaunchKernelGGL(k_r_reduce, dim3(nrhs), dim3(256), 0, st, r64 + P.r_part, nb, nrhs, out, gate);
  const int64_t gpart = P.r_part + P.r_nblk * P.max_rhs;
  hipLaunchKernelGGL(k_r_gsum<float>, dim3(nb), dim3(256), 0, st, k, nrhs, gpart);
  hipLaunchKernelGGL(k_r_reduce, dim3(nrhs), dim3(256), 0, st, r64 + gpart, nb, nrhs, out + P.max_rhs, gate);
  return hipGetLastError();
}
int *refine_ctl(const Plan &P, uint8_t *ws) { return (int *)(ws + P.b_status) + 16; }
const double *refine_rel(const Plan &P, uint8_t *ws) { return (const double *)(ws + P.b_r64) + P.r_ctl; }
hipError_t refine_ctl_reset(const Plan &P, uint8_t *ws, hipStream_t st) {
  hipLaunchKernelGGL(k_r_ctl_reset, dim3(1), dim3(64), 0, st, refine_ctl(P, ws));
  return hipGetLastError();
}
hipError_t refine_test(const Plan &P, uint8_t *ws, int nrhs, double tol, bool count, hipStream_t st) {
  double *r64 = (double *)(ws + P.b_r64);
  hipLaunchKernelGGL(k_r_test, dim3(1), dim3(256), 0, st, r64 + P.r_norm, r64 + P.r_fnorm, nrhs, (int)P.max_rhs, tol,
                     refine_ctl(P, ws), r64 + P.r_ctl, count ? 1 : 0);
  return hipGetLastError();
}
hipError_t refine_out(const Plan &P, uint8_t *ws, void *u, int64_t ldu, void *lam, int64_t ldl, int nrhs,
                      hipStream_t st) {
  KP<float> k = make_kp<float>(P, ws, ws + P.b_vals);
  if (P.n_torn > 0)
    hipLaunchKernelGGL(k_r_uout<float>, dim3((unsigned)((P.n_torn + 63) / 64), (unsigned)((nrhs + 7) / 8)),
                       dim3(256), 0, st, k, (cd *)u, ldu, nrhs);
  if (lam && P.n_mult > 0)
    hipLaunchKernelGGL(k_r_lout<float>, dim3(nblk(P.n_mult * nrhs)), dim3(256), 0, st, k, (cd *)lam, ldl, nrhs);
  return hipGetLastError();
}

}  // namespace dd
