// Internal data layout shared by the host planner and the HIP kernels.
//
// Every front (dense frontal matrix of the multifrontal LDL^T) is factored
// column-major, planar complex: the real plane at `off`, the imaginary plane
// at `off + n*n` (elements of the factor precision T).  Only the lower
// triangle is meaningful; after the pivot-tile factorisation the strict lower
// triangle of every diagonal NB x NB tile holds L11^-1 (not L11).  The full
// front lives only while it is factored and until its parent has gathered
// its update block; its first s columns (the factor) are then kept at `loff`
// (real plane n x s, imaginary plane after it) unless the front has no
// update block (loff = off).
#pragma once
#include <cstdint>

namespace dd {

constexpr int NB = 64;        // pivot-tile width of the blocked LDL^T
constexpr int GT = 64;        // output tile edge of the MFMA GEMMs
constexpr int KBLK = 256;     // outer block (columns per trailing update)
// fronts up to this size are substituted by one workgroup; wider ones carry
// Z = L11^-1 and use the split products (measured faster from 64 up, with 8
// and with 64 right-hand sides)
constexpr int FUSE_N = 64;
constexpr int ZKC = 256;      // K chunk of the split substitution products
constexpr int ZMMA_MIN = 8;   // above this many right-hand sides they run on MFMA

enum FrontKind : int32_t { FK_INTERIOR = 0, FK_GAMMA = 1, FK_AUX = 2 };

struct FrontDev {
  int64_t off;     // front matrix (T elements), ld = n, imaginary plane at off + n*n;
                   // while the front's level (and its parent's) is factored
  int64_t loff;    // stored factor read by the solves: columns [0, s) with ld n,
                   // imaginary plane at loff + lpim (FK_GAMMA: -1, the solves use X)
  int64_t lpim;
  int64_t woff;    // W scratch (T elements): re plane [n x wcols], im plane after it
  int64_t soff;    // index of fully-summed position 0 in the side arrays
  int64_t voff;    // solve vector (T elements): re plane [n x max_rhs], im after it
  int64_t xoff;    // FK_GAMMA: interface inverse X (T elements), g x g planar; else -1
  int64_t goff;    // FK_GAMMA: two g x max_rhs planar vectors (YG then h); else -1
  int64_t idx;     // first entry of this front's variable list in the index array
  int64_t vbase;   // row base of the front's variables in the global vector
  int64_t child;   // first entry in the child arrays
  int32_t n, s;    // front size, fully-summed count
  int32_t nchild;
  int32_t kind;
  int32_t dom;     // owning domain (aux: -1)
  int32_t wcols;   // columns of one W scratch buffer
  int64_t wstride; // fronts with more than one outer block: offset (T elements) of the
                   // second W buffer, used by odd outer blocks; else 0
  int64_t uoff;    // entry of update row s in the parent-row map (rows s..n-1 follow)
  int32_t parent;  // parent front (-1: none; then n == s)
  int32_t upad;
};

// Work item of one workgroup; the meaning of k, i, j depends on the kernel.
struct Item {
  int32_t f, k, i, j;
};

// Original entry of a domain matrix: value index -> position inside a front.
struct SPair {
  int64_t src;   // index in the concatenated value array
  int32_t pos;   // r + c*n inside the front (r >= c)
  int32_t pad;
};

// One dense block pair of an auxiliary front filled from interface inverses:
// front(pb + j, pa + i) += sum_d sa_d[i] sb_d[j] X_d(gb_d[j], ga_d[i]).
struct AuxItem {
  int32_t f;
  int32_t pa, pb;
  int32_t na, nb;
  int32_t ndom;
  int32_t same;
  int32_t pad;
  int64_t xoff[2];
  int64_t ga[2], gb[2];    // offsets into the (gpos, gsign) arrays
  int32_t g[2];
};

// The two entries of one multiplier: (offset of the interface value in the
// YG buffer of the domain, leading dimension of that buffer, sign) and the
// torn rows (for the FP64 residual).
struct MultRef {
  int64_t o[2];
  int64_t row[2];
  int32_t g[2];
  int32_t sg[2];
};

// One interface position of a domain: where its h value goes, and the range
// of multipliers acting on it.
struct GamRef {
  int64_t o;       // offset of the position inside the h buffer (column 0)
  int32_t g;       // leading dimension of that buffer
  int32_t beg, cnt;
  int32_t pad;
};

}  // namespace dd
