// HIP kernels of libspx for gfx950 (MI355X): tile packing, the persistent task-graph
// scheduler, and the FP64 tile kernels of the Cholesky factorisation and solve.
//
// Task model (Specx Sec. 2.1, Sec. 4.5, Sec. 4.7): the host inserts tasks in program
// order and turns their declared accesses into successor lists.  One persistent kernel
// runs the whole graph: every workgroup loops pop -> run -> release.  A task whose
// predecessors have all finished is pushed into a ready queue; an idle workgroup pops
// the highest non-empty priority level; when a task finishes, each successor's counter
// of unfinished predecessors is decremented atomically and the one that reaches zero is
// pushed.  Large tasks are cut into parts (row strips or 128x128 sub-blocks) that
// different workgroups run at the same time; the task counts as finished when its last
// part does.
#include <hip/hip_runtime.h>

#include <climits>
#include <mutex>

#include "spx_internal.h"

namespace spx {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef unsigned long long u64;

// Global-memory views of the generic pointers the tile kernels receive.  Loads through
// them compile to global_* instructions, which count only on vmcnt; generic (flat) loads
// also count on lgkmcnt, so every wait for an LDS read would wait for them too.
#define GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const GLOBAL T* gp(const T* p) {
  return (const GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ GLOBAL T* gp(T* p) {
  return (GLOBAL T*)p;
}
// LDS views of the generic pointers to the workgroup's shared buffer: in functions the
// compiler keeps out of line it would otherwise rebuild every LDS address from the 64-bit
// generic pointer (with a null check) at each access.
#define LDSAS __attribute__((address_space(3)))
template <class T>
__device__ __forceinline__ const LDSAS T* lp(const T* p) {
  return (const LDSAS T*)p;
}
template <class T>
__device__ __forceinline__ LDSAS T* lp(T* p) {
  return (LDSAS T*)p;
}

constexpr int NT = 256;                 // threads per workgroup (4 waves)
constexpr int LDS_DOUBLES = 16384;      // 128 KiB of LDS per workgroup (one workgroup per CU)
constexpr int LDS_D_OFF = 8192;         // 32x32 diagonal block, after the update staging area
constexpr u64 EMPTY = ~0ull;
constexpr uint32_t EMPTY32 = ~0u;

__device__ __forceinline__ double* tile_ptr(const DevMat& m, int i, int j) {
  return m.tiles + ((size_t)i * (size_t)(i + 1) / 2 + (size_t)j) * (size_t)m.b * (size_t)m.b;
}

__device__ __forceinline__ u64 now_ticks() { return wall_clock64(); }

// Inverses of the 32x32 diagonal blocks of diagonal tile k: b/32 column-major blocks.
__device__ __forceinline__ double* dinv_ptr(const DevMat& m, int k) { return m.dinv + (size_t)k * 32 * m.b; }
// Rows (and columns) of tile row k that hold the matrix, rounded up to 32: the rest of the
// last tile row is identity padding.
__device__ __forceinline__ int tile_active(const DevMat& m, int k) {
  const int rem = m.n - k * m.b;
  return rem >= m.b ? m.b : ((rem + 31) & ~31);
}

// Relaxed agent-scope load of a scheduler counter (ordering comes from explicit fences).
__device__ __forceinline__ uint32_t ld_rlx(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Epilogue of the 2x2-wave updates, C -= acc over a wave's NB x NB blocks of 16 x 16.  The
// products are formed transposed (the B fragment is the matrix core's first operand), so
// lane l holds rows row0 + 16 i + l%16 of C: sixteen lanes cover sixteen consecutive
// doubles of one column.  Element v of the accumulator is column col0 + 16 j + cofs(l, v):
// (l/16 + 4v) for the FP64 form, (4(l/16) + v) for the FP32-accumulating forms.  Every old
// value is loaded before any is stored, so the loads overlap.  sgn = 1 subtracts the
// product; sgn = -1 adds it (sgn * acc is exact, so both round once, as C - acc / C + acc).
template <int NB, bool F64_LAYOUT, class ACC>
__device__ __forceinline__ void update_epilogue(double* C, int ldc, const ACC (&acc)[NB][NB], int row0, int col0,
                                                int M, int N, bool lower, double sgn = 1.0) {
  const int lane = threadIdx.x & 63;
  GLOBAL double* Cg = gp(C);
  double old[NB][NB][4];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + i * 16 + (lane & 15);
        const int col = col0 + j * 16 + (F64_LAYOUT ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v);
        old[i][j][v] = (row < M && col < N && (!lower || row >= col)) ? Cg[(size_t)col * ldc + row] : 0.0;
      }
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + i * 16 + (lane & 15);
        const int col = col0 + j * 16 + (F64_LAYOUT ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v);
        if (row < M && col < N && (!lower || row >= col))
          Cg[(size_t)col * ldc + row] = old[i][j][v] - sgn * (double)acc[i][j][v];
      }
}

// ---------------------------------------------------------------------------------------
// FP64 matrix-core update: C[M x N] -= A[M x K] * B[N x K]^T (all column-major).
// Four waves in a 2x2 arrangement, each owning a WT x WT block of C made of 16x16
// v_mfma_f64_16x16x4 accumulators.  K is staged through LDS in chunks of 32, double
// buffered: while chunk c is multiplied out of one buffer, chunk c+1 (loaded into
// registers during the previous chunk) is written to the other and chunk c+2's global
// loads are issued, so each chunk needs one barrier and its loads have a whole chunk of
// matrix-core work to arrive.  M, N: multiples of 16, at most 2*WT.  K: multiple of 32.
// lower: write only the entries with row >= col (diagonal blocks of a symmetric update).
// FULL (M = N = 2*WT): the chunk loads carry no row guard, so a chunk's loads issue back to
// back with no branch between them (measured on one CU: 96 -> 81 us per 128x128x512 part;
// 167 -> 127 us when every part streams its operands).  Only the tiled-product kernel uses
// it: in the Cholesky kernel its extra registers made the compiler spill (see run_part).
// ---------------------------------------------------------------------------------------
template <int WT, bool FULL = false>
__device__ __forceinline__ void gemm_nt_f64(double* __restrict__ C, int ldc, const double* __restrict__ A, int lda,
                            const double* __restrict__ B, int ldb, int M, int N, int K, bool lower,
                            double* __restrict__ lds, double sgn = 1.0) {
  constexpr int SB = 2 * WT;
  constexpr int KC = 32;
  constexpr int NB = WT / 16;
  constexpr int PAIRS = SB * KC / (2 * NT);  // double2 loads per thread per operand
  constexpr int BUF = 2 * KC * SB;           // one buffer: the A and B chunks
  static_assert(PAIRS >= 1, "tile too small for one double2 per thread");
  static_assert(2 * BUF <= LDS_DOUBLES, "two chunk buffers must fit in LDS");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  d4 acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  d2 ra[PAIRS], rb[PAIRS];
  auto gload = [&](int k0) {
    const GLOBAL double* Ak = gp(A) + (size_t)k0 * lda;
    const GLOBAL double* Bk = gp(B) + (size_t)k0 * ldb;
#pragma unroll
    for (int p = 0; p < PAIRS; ++p) {
      const int e = (tid + p * NT) * 2;
      const int m = e / SB, r = e % SB;
      ra[p] = (FULL || r < M) ? *(const GLOBAL d2*)(Ak + m * lda + r) : d2{0.0, 0.0};
      rb[p] = (FULL || r < N) ? *(const GLOBAL d2*)(Bk + m * ldb + r) : d2{0.0, 0.0};
    }
  };
  auto lstore = [&](int buf) {
    LDSAS double* As = lp(lds) + buf * BUF;
    LDSAS double* Bs = As + KC * SB;
#pragma unroll
    for (int p = 0; p < PAIRS; ++p) {
      const int e = (tid + p * NT) * 2;
      *(LDSAS d2*)(As + e) = ra[p];
      *(LDSAS d2*)(Bs + e) = rb[p];
    }
  };
  const int nchunks = K / KC;
  gload(0);
  __syncthreads();  // LDS may still be read by the caller's previous step
  lstore(0);
  if (nchunks > 1) gload(KC);
  __syncthreads();
  const int arow = wr * WT + (lane & 15), bcol = wc * WT + (lane & 15), kl = lane >> 4;
  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunks) {
      lstore(buf ^ 1);                          // chunk c+1, loaded during chunk c-1
      if (c + 2 < nchunks) gload((c + 2) * KC);  // chunk c+2 in flight during chunk c
    }
    const LDSAS double* As = lp(lds) + buf * BUF;
    const LDSAS double* Bs = As + KC * SB;
    // fragments double-buffered in registers: those of the next 4-deep step are read
    // from LDS before this step's products are issued, so their latency is covered
    double a[2][NB], b[2][NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) a[0][i] = As[kl * SB + arow + i * 16];
#pragma unroll
    for (int j = 0; j < NB; ++j) b[0][j] = Bs[kl * SB + bcol + j * 16];
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int cb = (kk >> 2) & 1;
      if (kk + 4 < KC) {
#pragma unroll
        for (int i = 0; i < NB; ++i) a[cb ^ 1][i] = As[(kk + 4 + kl) * SB + arow + i * 16];
#pragma unroll
        for (int j = 0; j < NB; ++j) b[cb ^ 1][j] = Bs[(kk + 4 + kl) * SB + bcol + j * 16];
      }
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[cb][j], a[cb][i], acc[i][j], 0, 0, 0);
    }
    __syncthreads();  // buffer buf ^ 1 is written; buffer buf may be overwritten next
  }
  // accumulator layout of v_mfma_f64_16x16x4 (measured on gfx950): element v of lane l
  // holds (row l/16 + 4v, column l%16) of the 16x16 product, here (B A^T): C row l%16,
  // C column l/16 + 4v
  update_epilogue<NB, true>(C, ldc, acc, wr * WT, wc * WT, M, N, lower, sgn);
}

// Dispatch on the block size: M, N <= 128.
__device__ __forceinline__ void gemm_nt_any(double* C, int ldc, const double* A, int lda, const double* B, int ldb, int M, int N,
                            int K, bool lower, double* lds) {
  const int mx = M > N ? M : N;
  if (mx > 64)
    gemm_nt_f64<64>(C, ldc, A, lda, B, ldb, M, N, K, lower, lds);
  else if (mx > 32)
    gemm_nt_f64<32>(C, ldc, A, lda, B, ldb, M, N, K, lower, lds);
  else
    gemm_nt_f64<16>(C, ldc, A, lda, B, ldb, M, N, K, lower, lds);
}

// ---------------------------------------------------------------------------------------
// Mixed-precision updates: C (FP64) -= A * B^T with A, B low-precision copies of panel
// tiles, products accumulated in FP32 on the matrix cores.  Same 2x2-wave arrangement as
// the FP64 update.  M, N <= 2*WT (multiples of 16), K = tile size.
// ---------------------------------------------------------------------------------------
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

// FP32 copies, column-major (like the FP64 tiles); v_mfma_f32_16x16x4f32, whose result
// element v of lane l is (row 4*(l/16)+v, column l%16) of the 16x16 block.
template <int WT>
__device__ void gemm_nt_f32(double* __restrict__ C, int ldc, const float* __restrict__ A, int lda,
                            const float* __restrict__ B, int ldb, int M, int N, int K, bool lower,
                            double* __restrict__ lds_d) {
  constexpr int SB = 2 * WT, KC = 32, NB = WT / 16;
  constexpr int QUADS = SB * KC / (4 * NT);  // float4 loads per thread per operand
  static_assert(QUADS >= 1, "tile too small");
  LDSAS float* As = lp(reinterpret_cast<float*>(lds_d));
  LDSAS float* Bs = As + KC * SB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  f4 acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  f4 ra[QUADS], rb[QUADS];
  auto gload = [&](int k0) {
#pragma unroll
    for (int p = 0; p < QUADS; ++p) {
      const int e = (tid + p * NT) * 4;
      const int m = e / SB, r = e % SB;
      ra[p] = (r < M) ? *(const GLOBAL f4*)(gp(A) + (size_t)(k0 + m) * lda + r) : f4{0.f, 0.f, 0.f, 0.f};
      rb[p] = (r < N) ? *(const GLOBAL f4*)(gp(B) + (size_t)(k0 + m) * ldb + r) : f4{0.f, 0.f, 0.f, 0.f};
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int p = 0; p < QUADS; ++p) {
      const int e = (tid + p * NT) * 4;
      *(LDSAS f4*)(As + e) = ra[p];
      *(LDSAS f4*)(Bs + e) = rb[p];
    }
  };
  const int nchunks = K / KC;
  gload(0);
  __syncthreads();
  lstore();
  __syncthreads();
  const int arow = wr * WT + (lane & 15), bcol = wc * WT + (lane & 15), kl = lane >> 4;
  for (int c = 0; c < nchunks; ++c) {
    if (c + 1 < nchunks) gload((c + 1) * KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      float a[NB], bq[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) a[i] = As[(kk + kl) * SB + arow + i * 16];
#pragma unroll
      for (int j = 0; j < NB; ++j) bq[j] = Bs[(kk + kl) * SB + bcol + j * 16];
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bq[j], a[i], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
    if (c + 1 < nchunks) {
      lstore();
      __syncthreads();
    }
  }
  update_epilogue<NB, false>(C, ldc, acc, wr * WT, wc * WT, M, N, lower);  // transposed product
}

// BF16 copies, row-major inside the tile (element (r, k) at r*ld + k) so that the eight
// consecutive k a lane feeds to v_mfma_f32_16x16x32_bf16 are contiguous: lane l supplies
// A[l%16][8(l/16) .. 8(l/16)+7] and B^T likewise; result layout as for the FP32 form.
template <int WT>
__device__ void gemm_nt_bf16(double* __restrict__ C, int ldc, const uint16_t* __restrict__ A, int lda,
                             const uint16_t* __restrict__ B, int ldb, int M, int N, int K, bool lower,
                             double* __restrict__ lds_d) {
  constexpr int SB = 2 * WT, KC = 32, NB = WT / 16, LS = KC + 8;  // padded LDS row
  constexpr int CH = SB * (KC / 8);                                 // 16-byte chunks per operand
  constexpr int PER = (CH + NT - 1) / NT;
  LDSAS uint16_t* As = lp(reinterpret_cast<uint16_t*>(lds_d));
  LDSAS uint16_t* Bs = As + SB * LS;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  f4 acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  u4 ra[PER], rb[PER];
  auto gload = [&](int k0) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = tid + p * NT;  // chunk: row e / 4, k offset 8 (e % 4)
      const int r = e >> 2, kq = (e & 3) * 8;
      const u4 z = {0u, 0u, 0u, 0u};
      ra[p] = (e < CH && r < M) ? *(const GLOBAL u4*)(gp(A) + (size_t)r * lda + k0 + kq) : z;
      rb[p] = (e < CH && r < N) ? *(const GLOBAL u4*)(gp(B) + (size_t)r * ldb + k0 + kq) : z;
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = tid + p * NT;
      if (e < CH) {
        const int r = e >> 2, kq = (e & 3) * 8;
        *(LDSAS u4*)(As + r * LS + kq) = ra[p];
        *(LDSAS u4*)(Bs + r * LS + kq) = rb[p];
      }
    }
  };
  const int nchunks = K / KC;
  gload(0);
  __syncthreads();
  lstore();
  __syncthreads();
  const int arow = wr * WT + (lane & 15), bcol = wc * WT + (lane & 15), kq = 8 * (lane >> 4);
  for (int c = 0; c < nchunks; ++c) {
    if (c + 1 < nchunks) gload((c + 1) * KC);
    bf8 a[NB], bq[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) a[i] = __builtin_bit_cast(bf8, *(const LDSAS u4*)(As + (arow + i * 16) * LS + kq));
#pragma unroll
    for (int j = 0; j < NB; ++j) bq[j] = __builtin_bit_cast(bf8, *(const LDSAS u4*)(Bs + (bcol + j * 16) * LS + kq));
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bq[j], a[i], acc[i][j], 0, 0, 0);
    __syncthreads();
    if (c + 1 < nchunks) {
      lstore();
      __syncthreads();
    }
  }
  update_epilogue<NB, false>(C, ldc, acc, wr * WT, wc * WT, M, N, lower);  // transposed product
}

// FP64 -> BF16, round to nearest even, directly from the double (no intermediate FP32
// rounding).  Magnitudes below the FP32 normal range flush to a signed zero.
__device__ __forceinline__ uint16_t to_bf16(double x) {
  unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const unsigned long long sign = u >> 63;
  u &= 0x7fffffffffffffffull;
  if (u >= 0x7ff0000000000000ull) return (uint16_t)((sign << 15) | 0x7f80u | (u > 0x7ff0000000000000ull ? 0x40u : 0u));
  const unsigned long long lsb = (u >> 45) & 1ull;
  u += (1ull << 44) - 1ull + lsb;  // 45 dropped bits: round half to even
  const int e = (int)(u >> 52) - 1023 + 127;
  if (e <= 0) return (uint16_t)(sign << 15);
  if (e >= 255) return (uint16_t)((sign << 15) | 0x7f80u);
  return (uint16_t)((sign << 15) | ((unsigned)e << 7) | (unsigned)((u >> 45) & 0x7fu));
}

// Orders a wave's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave writes Z = L^{-1} for a factored 32x32 lower block L (LDS, column-major, zeros
// above the diagonal): lane c forward-substitutes L z = e_c, reading the entries of L as
// same-address LDS loads (broadcasts).  The reciprocals of the diagonal are made first, in
// parallel, so the substitution chain holds only multiplications and FMAs.  Z may not be L.
__device__ void lower_inverse32(const double* __restrict__ Lg, double* __restrict__ Zg) {
  const int lane = threadIdx.x & 63;
  const LDSAS double* L = lp(Lg);
  LDSAS double* Z = lp(Zg);
  LDSAS double* R = Z;  // the 32 reciprocals, in Z until Z is written
  if (lane < 32) R[lane] = 1.0 / L[lane * 33];
  wave_lds_sync();
  double z[32];
#pragma unroll
  for (int m = 0; m < 32; ++m) z[m] = (m == lane) ? 1.0 : 0.0;
  // software pipeline: column p + 1 of L (and its reciprocal pivot) is loaded while column
  // p is applied, so the LDS latency overlaps the substitution
  double cn[32], rn = R[0];
#pragma unroll
  for (int m = 1; m < 32; ++m) cn[m] = L[m];
#pragma unroll
  for (int p = 0; p < 32; ++p) {
    double cc[32];
    const double rp = rn;
#pragma unroll
    for (int m = p + 1; m < 32; ++m) cc[m] = cn[m];
    if (p + 1 < 32) {
      rn = R[p + 1];
#pragma unroll
      for (int m = p + 2; m < 32; ++m) cn[m] = L[(p + 1) * 32 + m];
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of this column's arithmetic
    z[p] *= rp;
#pragma unroll
    for (int m = p + 1; m < 32; ++m) z[m] -= cc[m] * z[p];
  }
  wave_lds_sync();  // every read of R is done
  if (lane < 32) {
#pragma unroll
    for (int m = 0; m < 32; ++m) Z[lane * 32 + m] = m >= lane ? z[m] : 0.0;
  }
}

// A double from one lane of the wave, as a uniform (scalar) value.
__device__ __forceinline__ double lane_value(double v, int l) {
  const unsigned long long u = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

// One wave factors the 32x32 lower block D (column-major in LDS, D(r, j) at D[j*32 + r]) in
// place and writes its inverse to Z (column-major, zeros above the diagonal), in one
// right-looking pass over the columns.  Lanes 0-31 hold row r of the block being factored,
// lanes 32-63 column r of Z = L^{-1} (starting from e_r); column c of L, once scaled, is
// applied by both halves alike (v[j] -= a L(j, c) for j > c, with a = L(r, c) in a factor
// lane and Z(c, r) in an inverse lane), so the inverse rides on the factorization's
// broadcasts.  The pivot and L(c+1, c) move between lanes as uniform values, and the rest
// of column c goes through LDS and is applied one column later, so the LDS round trip is
// off the pivot chain; every entry still takes its updates in column order.  Column scale
// r: the hardware reciprocal square root refined by two Newton steps, L(c, c) = p r (no
// IEEE square root).  Returns the 1-based column of the first non-positive or NaN pivot (D
// and Z then hold partial values), or 0; the same value in every lane.
__device__ __forceinline__ int factor_inverse32(double* __restrict__ Dg, double* __restrict__ Zg) {
  const int lane = threadIdx.x & 63, r = lane & 31;
  const bool inv = lane >= 32;
  LDSAS double* D = lp(Dg);
  LDSAS double* Z = lp(Zg);
  double v[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const double x = D[j * 32 + r];
    v[j] = inv ? (j == r ? 1.0 : 0.0) : (r >= j ? x : 0.0);
  }
  wave_lds_sync();  // every lane has read D before column 0 is overwritten
  double col[32];   // column c - 1 of L, rows c + 1 .. 31, from LDS
  double aprev = 0.0;
#pragma unroll
  for (int c = 0; c < 32; ++c) {
    const double p = lane_value(v[c], c);
    // a uniform branch; it also ends the column's basic block, which keeps the compiler
    // from sinking the column's updates to their last use
    if (!(p > 0.0)) return c + 1;
    const double hp = 0.5 * p;
    double rs = __builtin_amdgcn_rsq(p);
    rs = fma(rs, fma(-hp * rs, rs, 0.5), rs);
    rs = fma(rs, fma(-hp * rs, rs, 0.5), rs);
    // factor lanes: L(r, c) = v[c] rs below the diagonal and L(c, c) = p rs on it (v[c] = p
    // in lane c), 0 above; inverse lanes: Z(c, r) = v[c] / L(c, c) (0 for c < r), an IEEE
    // quotient as a substitution with the stored factor makes it
    const double af = r >= c ? v[c] * rs : 0.0;
    const double a = inv ? v[c] * (1.0 / (p * rs)) : af;
    v[c] = a;
    // row c + 1 first (the next pivot): column c - 1's update, then column c's, with
    // L(c + 1, c) taken from lane c + 1 (af: the quotient stays off the pivot chain); then
    // column c - 1 on the rows after it
    if (c >= 1 && c + 1 < 32) v[c + 1] -= aprev * col[c + 1];
    if (c + 1 < 32) v[c + 1] -= a * lane_value(af, c + 1);
    if (c >= 1) {
#pragma unroll
      for (int j = c + 2; j < 32; ++j) v[j] -= aprev * col[j];
    }
    // column c of L to LDS; the inverse lanes store theirs into Z, which the end
    // overwrites (an address select rather than a divergent branch)
    (inv ? Z : D)[c * 32 + r] = a;
    wave_lds_sync();
    const LDSAS d2* C2 = (const LDSAS d2*)(D + c * 32);
#pragma unroll
    for (int h = (c + 2) >> 1; h < 16; ++h) {
      const d2 t = C2[h];
      col[2 * h] = t[0];
      col[2 * h + 1] = t[1];
    }
    aprev = a;
  }
  if (inv) {
#pragma unroll
    for (int m = 0; m < 32; ++m) Z[r * 32 + m] = m >= r ? v[m] : 0.0;
  }
  wave_lds_sync();
  return 0;
}

// One wave inverts an already factored 32x32 lower block L (LDS, column-major) into Z.
__device__ void inverse32(const double* __restrict__ L, double* __restrict__ Z) { lower_inverse32(L, Z); }

// ---------------------------------------------------------------------------------------
// Tall FP64 update for the panel steps: C[M x 32] -= A[M x K] * B[32 x K]^T (column-major).
// The 16-row blocks of C go round-robin to the four waves (block q to wave q % 4), each
// wave keeping its blocks' two 16x16 accumulators per block in registers.  B (32 x 16 per
// chunk) is double-buffered in LDS; A fragments come straight from global memory, one chunk
// ahead in registers; the chunk is deeper when each wave has fewer row blocks, so every
// chunk carries enough matrix-core work to cover the next chunk's loads.  M: multiple of
// 16, at most 64 * NBMAX.  K: multiple of 64 / NBMAX (of 16 for NBMAX >= 8).
// lower: write only row >= col (C starts on the diagonal).  ASSIGN: C = A * B^T instead; C
// may then be A itself, since each wave reads all of its rows before writing them.  Ma
// (a multiple of 16): only rows below Ma are read and written; the work split and each
// computed row's arithmetic are those of the full M.
// ---------------------------------------------------------------------------------------
template <int NBMAX, bool ASSIGN>
__device__ __forceinline__ void gemm_tall32_f64(double* __restrict__ C, int ldc, const double* __restrict__ A, int lda,
                                const double* __restrict__ B, int ldb, int M, int K, bool lower,
                                double* __restrict__ lds, int Ma = 1 << 30) {
  constexpr int KC = NBMAX >= 8 ? 16 : (NBMAX >= 2 ? 32 : 64), KS = KC / 4;  // more depth for fewer blocks
  constexpr int BPT = KC * 32 / NT;                                            // B elements per thread
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nblk = (Ma < M ? Ma : M) >> 4, kl = lane >> 4, li = lane & 15;
  d4 acc[NBMAX][2];
#pragma unroll
  for (int t = 0; t < NBMAX; ++t) acc[t][0] = acc[t][1] = d4{0.0, 0.0, 0.0, 0.0};
  double an[NBMAX][KS], bn[BPT];
  auto aload = [&](int k0) {
#pragma unroll
    for (int t = 0; t < NBMAX; ++t) {
      const int q = wave + 4 * t;
#pragma unroll
      for (int s = 0; s < KS; ++s)
        an[t][s] = q < nblk ? gp(A)[(size_t)(k0 + 4 * s + kl) * lda + 16 * q + li] : 0.0;
    }
  };
  auto bload = [&](int k0) {  // element e = tid + 256 i of the KC x 32 chunk: (k = e / 32, j = e % 32)
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      const int e = tid + NT * i;
      bn[i] = gp(B)[(size_t)(k0 + (e >> 5)) * ldb + (e & 31)];
    }
  };
  auto bstore = [&](LDSAS double* dst) {
#pragma unroll
    for (int i = 0; i < BPT; ++i) dst[tid + NT * i] = bn[i];
  };
  const int nch = K / KC;
  aload(0);
  bload(0);
  __syncthreads();  // the caller's previous use of LDS is over
  bstore(lp(lds));
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    double acur[NBMAX][KS];
#pragma unroll
    for (int t = 0; t < NBMAX; ++t)
#pragma unroll
      for (int s = 0; s < KS; ++s) acur[t][s] = an[t][s];
    const LDSAS double* Bc = lp(lds) + (c & 1) * (KC * 32);
    if (c + 1 < nch) {
      aload((c + 1) * KC);
      bload((c + 1) * KC);
    }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const double b0 = Bc[(4 * s + kl) * 32 + li], b1 = Bc[(4 * s + kl) * 32 + 16 + li];
#pragma unroll
      for (int t = 0; t < NBMAX; ++t) {
        if (wave + 4 * t < nblk) {
          acc[t][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, acur[t][s], acc[t][0], 0, 0, 0);
          acc[t][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, acur[t][s], acc[t][1], 0, 0, 0);
        }
      }
    }
    if (c + 1 < nch) bstore(lp(lds) + ((c + 1) & 1) * (KC * 32));
    __syncthreads();
  }
  // FP64 accumulator layout (l/16 + 4v, l%16) of the transposed product (B A^T): lane l
  // holds C row 16q + l%16, column 16 jb + l/16 + 4v, so sixteen lanes cover sixteen
  // consecutive doubles.  Without ASSIGN every old value is loaded before any store.
  GLOBAL double* Cg = gp(C);
  double old[NBMAX][2][4];
  if (!ASSIGN) {
#pragma unroll
    for (int t = 0; t < NBMAX; ++t) {
      const int q = wave + 4 * t;
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * q + li, col = 16 * jb + kl + 4 * v;
          old[t][jb][v] = (q < nblk && (!lower || row >= col)) ? Cg[(size_t)col * ldc + row] : 0.0;
        }
    }
  }
#pragma unroll
  for (int t = 0; t < NBMAX; ++t) {
    const int q = wave + 4 * t;
    if (q >= nblk) continue;
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * q + li, col = 16 * jb + kl + 4 * v;
        if (lower && row < col) continue;
        if (ASSIGN)
          Cg[(size_t)col * ldc + row] = acc[t][jb][v];
        else
          Cg[(size_t)col * ldc + row] = old[t][jb][v] - acc[t][jb][v];
      }
  }
}

// Tall update for the POTRF panels: C[M x 32] -= A B^T, barrier-free in its main loop.
// The waves form 4/KS row groups of KS waves; the waves of a group split K (wave w: row
// group w / KS, K range (w % KS) K/KS ...), each taking up to NBW 16-row blocks of its
// group and loading its fragments straight from global memory a group of G 4-deep steps
// ahead (no LDS, no barrier in the loop, so the four waves drift freely and the latency
// of one wave's loads hides behind the others' products).  With KS > 1 the partial
// products meet in LDS and each wave reduces and writes a quarter of the 16x16 tiles.
// Products transposed as in gemm_tall32_f64 (lane l: row 16q + l%16, column 16 jb + l/16
// + 4v).  M: multiple of 16, at most 16 NBW 4/KS.  K: multiple of 16 G KS.  Ma (a
// multiple of 16): only rows below Ma are read and written, with the work split and the
// per-row arithmetic of the full M.
template <int NBW, int G, int KS>
__device__ __forceinline__ void gemm_tall32_split(double* __restrict__ C, int ldc, const double* __restrict__ A, int lda,
                                  const double* __restrict__ B, int ldb, int M, int K, bool lower,
                                  double* __restrict__ lds, int Ma = 1 << 30) {
  constexpr int GROUPS = 4 / KS;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nblk = M >> 4, kl = lane >> 4, li = lane & 15;
  const int nbp = (nblk + GROUPS - 1) / GROUPS;  // row blocks per group
  const int rg = wave / KS, q0 = rg * nbp;
  const int nlive = (Ma < M ? Ma : M) >> 4;  // row blocks read and written
  const int nmine = nlive - q0 < nbp ? (nlive - q0 > 0 ? nlive - q0 : 0) : nbp;
  const int kq = K / KS, kb = (wave % KS) * kq;
  const GLOBAL double* Ag = gp(A);
  const GLOBAL double* Bg = gp(B);
  d4 acc[NBW][2];
#pragma unroll
  for (int t = 0; t < NBW; ++t) acc[t][0] = acc[t][1] = d4{0.0, 0.0, 0.0, 0.0};
  double an[G][NBW], bn[G][2];
  auto load = [&](int k0) {
#pragma unroll
    for (int s4 = 0; s4 < G; ++s4) {
      const size_t kr = (size_t)(k0 + 4 * s4 + kl);
#pragma unroll
      for (int t = 0; t < NBW; ++t) an[s4][t] = t < nmine ? Ag[kr * lda + 16 * (q0 + t) + li] : 0.0;
      bn[s4][0] = Bg[kr * ldb + li];
      bn[s4][1] = Bg[kr * ldb + 16 + li];
    }
  };
  const int ng = kq / (4 * G);
  if (ng > 0) load(kb);
  for (int g = 0; g < ng; ++g) {
    double ac[G][NBW], bc[G][2];
#pragma unroll
    for (int s4 = 0; s4 < G; ++s4) {
#pragma unroll
      for (int t = 0; t < NBW; ++t) ac[s4][t] = an[s4][t];
      bc[s4][0] = bn[s4][0];
      bc[s4][1] = bn[s4][1];
    }
    if (g + 1 < ng) load(kb + (g + 1) * 4 * G);
#pragma unroll
    for (int s4 = 0; s4 < G; ++s4)
#pragma unroll
      for (int t = 0; t < NBW; ++t) {
        if (t < nmine) {
          acc[t][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(bc[s4][0], ac[s4][t], acc[t][0], 0, 0, 0);
          acc[t][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(bc[s4][1], ac[s4][t], acc[t][1], 0, 0, 0);
        }
      }
  }
  GLOBAL double* Cg = gp(C);
  if (KS == 1) {  // each wave owns its rows: write them directly, all old values first
    double old[NBW][2][4];
#pragma unroll
    for (int t = 0; t < NBW; ++t)
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * (q0 + t) + li, col = 16 * jb + kl + 4 * v;
          old[t][jb][v] = (t < nmine && (!lower || row >= col)) ? Cg[(size_t)col * ldc + row] : 0.0;
        }
#pragma unroll
    for (int t = 0; t < NBW; ++t) {
      if (t >= nmine) continue;
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * (q0 + t) + li, col = 16 * jb + kl + 4 * v;
          if (!lower || row >= col) Cg[(size_t)col * ldc + row] = old[t][jb][v] - acc[t][jb][v];
        }
    }
    return;
  }
  // partials: P[w][tile][v][lane], tile = 2 t + jb of the wave's row group
  LDSAS double* P = lp(lds);
  constexpr int T = 2 * NBW;
  __syncthreads();  // the caller's previous use of LDS is over
#pragma unroll
  for (int t = 0; t < NBW; ++t)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v) P[((wave * T + 2 * t + jb) * 4 + v) * 64 + lane] = acc[t][jb][v];
  __syncthreads();
  for (int tile = wave; tile < 2 * nlive; tile += 4) {
    const int q = tile >> 1, jb = tile & 1;
    const int g0 = (q / nbp) * KS, lt = 2 * (q % nbp) + jb;  // first wave of the row group, its tile
    const int row = 16 * q + li;
    double sum[4], old[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double acc_v = 0.0;
#pragma unroll
      for (int h = 0; h < KS; ++h) acc_v += P[(((g0 + h) * T + lt) * 4 + v) * 64 + lane];
      sum[v] = acc_v;
      const int col = 16 * jb + kl + 4 * v;
      old[v] = (!lower || row >= col) ? Cg[(size_t)col * ldc + row] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int col = 16 * jb + kl + 4 * v;
      if (!lower || row >= col) Cg[(size_t)col * ldc + row] = old[v] - sum[v];
    }
  }
  __syncthreads();  // LDS partials consumed before the caller reuses LDS
}

__device__ __forceinline__ void gemm_tall32_any(double* C, int ldc, const double* A, int lda, const double* B, int ldb, int M, int K,
                                bool lower, double* lds, int Ma = 1 << 30) {
  if (K <= 0 || M <= 0) return;
  if (M <= 128 && K % 64 == 0) {  // few rows: K split four ways
    if (M <= 32) gemm_tall32_split<2, 4, 4>(C, ldc, A, lda, B, ldb, M, K, lower, lds, Ma);
    else if (M <= 64) gemm_tall32_split<4, 4, 4>(C, ldc, A, lda, B, ldb, M, K, lower, lds, Ma);
    else gemm_tall32_split<8, 4, 4>(C, ldc, A, lda, B, ldb, M, K, lower, lds, Ma);
  } else if (M <= 128 && K % 32 == 0) {
    if (M <= 32) gemm_tall32_split<2, 2, 4>(C, ldc, A, lda, B, ldb, M, K, lower, lds, Ma);
    else if (M <= 64) gemm_tall32_split<4, 2, 4>(C, ldc, A, lda, B, ldb, M, K, lower, lds, Ma);
    else gemm_tall32_split<8, 2, 4>(C, ldc, A, lda, B, ldb, M, K, lower, lds, Ma);
  } else if (M <= 256 && K % 32 == 0) {  // two row groups, K split two ways
    gemm_tall32_split<8, 4, 2>(C, ldc, A, lda, B, ldb, M, K, lower, lds, Ma);
  } else if (M <= 512 && K % 16 == 0) {  // four row groups
    gemm_tall32_split<8, 4, 1>(C, ldc, A, lda, B, ldb, M, K, lower, lds, Ma);
  } else if (M <= 64 && K % 64 == 0) {
    gemm_tall32_f64<1, false>(C, ldc, A, lda, B, ldb, M, K, lower, lds, Ma);
  } else if (M <= 128 && K % 32 == 0) {
    gemm_tall32_f64<2, false>(C, ldc, A, lda, B, ldb, M, K, lower, lds, Ma);
  } else if (M <= 256 && K % 32 == 0) {
    gemm_tall32_f64<4, false>(C, ldc, A, lda, B, ldb, M, K, lower, lds, Ma);
  } else {
    gemm_tall32_f64<8, false>(C, ldc, A, lda, B, ldb, M, K, lower, lds, Ma);
  }
}

// X[M x 32] <- X * Li^T in place, Li a 32x32 block inverse (column-major, ld 32); rows
// from Ma on are left alone.
__device__ __forceinline__ void apply_inv_tall(double* X, int ldx, const double* Li, int M, double* lds,
                                               int Ma = 1 << 30) {
  if (M <= 0 || Ma <= 0) return;
  if (M <= 128)
    gemm_tall32_f64<2, true>(X, ldx, X, ldx, Li, 32, M, 32, false, lds, Ma);
  else
    gemm_tall32_f64<8, true>(X, ldx, X, ldx, Li, 32, M, 32, false, lds, Ma);
}

// One workgroup factors the updated 32x32 diagonal block at (c0, c0) of a b x b tile in
// place (one wave, in LDS) and stores its inverse as block c0/32 of dinv.  Returns (to all
// threads) 0 or the 1-based local column of a non-positive or NaN pivot.
__device__ __forceinline__ int factor_diag32(double* __restrict__ a, int b, int c0, double* __restrict__ dinv,
                             double* __restrict__ lds) {
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  double* D = lds + LDS_D_OFF;
  double* Z = D + 1024;
  LDSAS double* Dl = lp(D);
  LDSAS double* Zl = lp(Z);
  for (int e = tid; e < 1024; e += NT) {
    const int r = e & 31, j = e >> 5;
    Dl[e] = r >= j ? a[(size_t)(c0 + j) * b + c0 + r] : 0.0;
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();
  if (tid < 64) {
    const int bad = factor_inverse32(D, Z);
    if (bad && tid == 0) s_bad = c0 + bad;
  }
  __syncthreads();
  if (s_bad) return s_bad;
  double* dblk = dinv + (size_t)c0 * 32;
  for (int e = tid; e < 1024; e += NT) {
    const int r = e & 31, j = e >> 5;
    if (r >= j) a[(size_t)(c0 + j) * b + c0 + r] = Dl[e];
    dblk[e] = Zl[e];
  }
  __syncthreads();
  return 0;
}

// ---------------------------------------------------------------------------------------
// POTRF: in-place lower Cholesky of one b x b tile by one workgroup.  Left-looking over
// 32-wide panels: the panel (rows c0.., columns c0..c0+31) first receives the updates of
// every factored column (tall matrix-core update, K = c0); one wave then factors its 32x32
// diagonal block in LDS and inverts it; the rows below are multiplied by the transposed
// inverse on the matrix cores (K = 32).  The inverses of the diagonal blocks are stored in
// dinv (b/32 column-major 32x32 blocks) for the TRSM and solve tasks.  na (a multiple of
// 32): the tile's rows and columns from na on are the identity padding of the matrix's
// last tile, which factors to itself: they are not touched, and their diagonal blocks'
// inverses are written as identities.  The rows below na take exactly the arithmetic of
// the full tile (the update kernels are chosen by the full row count).  Returns (to all
// threads) 0 or the 1-based local column of a non-positive or NaN pivot.
// ---------------------------------------------------------------------------------------
__device__ __noinline__ int potrf_tile(double* __restrict__ a, int b, double* __restrict__ dinv, double* __restrict__ lds,
                                       int na) {
  for (int c0 = 0; c0 < na; c0 += 32) {
    gemm_tall32_any(a + (size_t)c0 * b + c0, b, a + c0, b, a + c0, b, b - c0, c0, true, lds, na - c0);
    __syncthreads();
    const int bad = factor_diag32(a, b, c0, dinv, lds);
    if (bad) return bad;
    apply_inv_tall(a + (size_t)c0 * b + c0 + 32, b, dinv + (size_t)c0 * 32, b - c0 - 32, lds, na - c0 - 32);
    __syncthreads();
  }
  for (int e = threadIdx.x; e < (b - na) * 32; e += NT) dinv[(size_t)na * 32 + e] = ((e & 31) == ((e >> 5) & 31)) ? 1.0 : 0.0;
  return 0;
}

// ---------------------------------------------------------------------------------------
// POTRF split into b/32 dependent steps, each cut into workgroup parts, for the large
// diagonal tiles whose single-workgroup factorization would hold up the whole
// elimination.  The algorithm is the left-looking one above, with the scaling of a
// column block by the inverse of its diagonal block deferred to the next step, so one
// step needs no wait inside it.  Step c (c0 = 32 c), with 32-row blocks R_r:
//   part 0:  R_{c+1}[:, c-1] <- R_{c+1}[:, c-1] Z_{c-1}^T   (if c >= 1 and c + 1 < b/32)
//            (R_c; R_{c+1})[:, c] -= (R_c; R_{c+1})[:, 0:c0] R_c[:, 0:c0]^T
//            factor and invert the diagonal block (c, c) -> L_cc, Z_c
//            R_{c+1}[:, c] <- R_{c+1}[:, c] Z_c^T
//   part p >= 1 (c >= 1), r = c + 1 + p:
//            R_r[:, c-1] <- R_r[:, c-1] Z_{c-1}^T
//            R_r[:, c] -= R_r[:, 0:c0] R_c[:, 0:c0]^T
// Every block R_c[:, 0:c0] read by the row parts was made final in an earlier step, and
// part 0 writes only row blocks c and c + 1, which no row part reads, so the parts of a
// step are independent; successive steps are ordered by the task graph.  The update of a
// row block may split K differently from potrf_tile's (its kernel depends on the row
// count), so the two forms agree to rounding, not bitwise.  na: as for potrf_tile, rows
// and columns from na on are identity padding; the steps and row blocks there only write
// identity block inverses.  Returns (to all threads) 0 or the 1-based local column of a
// bad pivot.
// ---------------------------------------------------------------------------------------
__device__ __noinline__ int potrf_step_part(double* __restrict__ a, int b, double* __restrict__ dinv, int c, int part,
                                            double* __restrict__ lds, int na) {
  const int nb = b >> 5, c0 = 32 * c;
  if (part > 0) {
    const int r0 = 32 * (c + 1 + part);
    if (c < 1 || r0 >= na) return 0;
    apply_inv_tall(a + (size_t)(c0 - 32) * b + r0, b, dinv + (size_t)(c0 - 32) * 32, 32, lds);
    __syncthreads();
    gemm_tall32_any(a + (size_t)c0 * b + r0, b, a + r0, b, a + c0, b, 32, c0, false, lds);
    return 0;
  }
  if (c0 >= na) {  // a step of the identity padding: its block inverse is the identity
    for (int e = threadIdx.x; e < 1024; e += NT) dinv[(size_t)c0 * 32 + e] = ((e & 31) == (e >> 5)) ? 1.0 : 0.0;
    return 0;
  }
  const bool look = c + 1 < nb;
  if (c >= 1 && look) {
    apply_inv_tall(a + (size_t)(c0 - 32) * b + c0 + 32, b, dinv + (size_t)(c0 - 32) * 32, 32, lds, na - c0 - 32);
    __syncthreads();
  }
  gemm_tall32_any(a + (size_t)c0 * b + c0, b, a + c0, b, a + c0, b, look ? 64 : 32, c0, true, lds, na - c0);
  __syncthreads();
  const int bad = factor_diag32(a, b, c0, dinv, lds);
  if (bad) return bad;
  if (look) apply_inv_tall(a + (size_t)c0 * b + c0 + 32, b, dinv + (size_t)c0 * 32, 32, lds, na - c0 - 32);
  return 0;
}

// ---------------------------------------------------------------------------------------
// TRSM part: rows [r0, r0+32) of an off-diagonal tile X <- X L^{-T}, L the factored diagonal
// tile of the same block column, dinv the inverses Li_c of its 32x32 diagonal blocks.
// Right-looking over 32-wide column blocks with the strip resident in matrix-core
// accumulators: 16-column block j of the strip belongs to wave j % 4, as two 16x16 tiles.
// The products are formed transposed (as in the updates), so a tile's accumulator element
// v in lane l is X(16 rb + l%16, 16 j + l/16 + 4v), which is also the operand layout of a
// 4-deep slice: the strip feeds the matrix cores without a transpose.  Step c: the owners
// of block c stage it in LDS, form X_c <- X_c Li_c^T and publish it (LDS, the tile, and in
// mixed precision the FP32 or BF16 copy the updates read); then every wave subtracts
// X_c L(j, c)^T from each of its later blocks j.  k0 (a multiple of 32): the strip's
// columns before k0 are zero and stay zero (the inversion task starts at its identity
// rows' diagonal); they are neither read nor written.
// ---------------------------------------------------------------------------------------
template <int NCB>
__device__ __forceinline__ void trsm_strip32(double* __restrict__ x, const double* __restrict__ l, const double* __restrict__ dinv,
                             int b, int r0, void* __restrict__ low, int prec, double* __restrict__ lds, int k0) {
  constexpr int LDX = 34;  // padded LDS column (32 rows)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, kl = lane >> 4;
  const int ncb = b / 16;
  LDSAS double* Xs = lp(lds);             // block c before its diagonal solve, column-major 32 x 32
  LDSAS double* Xn = lp(lds) + 32 * LDX;  // block c after it
  GLOBAL double* xg = gp(x) + r0;
  const GLOBAL double* lg = gp(l);
  d4 acc[2][NCB];
#pragma unroll
  for (int t = 0; t < NCB; ++t) {
    const int cb = wave + 4 * t;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        acc[rb][t][v] = (cb < ncb && 16 * cb >= k0) ? xg[(size_t)(16 * cb + kl + 4 * v) * b + 16 * rb + li] : 0.0;
  }
  __syncthreads();  // the caller's previous use of LDS is over
  for (int c0 = k0; c0 < b; c0 += 32) {
    const int cblk = c0 / 16;
    // (1) the owners of block c stage it
#pragma unroll
    for (int t = 0; t < NCB; ++t) {
      const int kb = wave + 4 * t - cblk;
      if (kb == 0 || kb == 1) {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int v = 0; v < 4; ++v) Xs[(16 * kb + kl + 4 * v) * LDX + 16 * rb + li] = acc[rb][t][v];
      }
    }
    __syncthreads();
    // (2) X_c Li^T: output 16-column half jb from both input halves kb (Li lower triangular,
    // so the upper input half does not reach the lower output half)
#pragma unroll
    for (int t = 0; t < NCB; ++t) {
      const int jb = wave + 4 * t - cblk;
      if (jb == 0 || jb == 1) {
        const GLOBAL double* Li = gp(dinv) + (size_t)c0 * 32;  // Li(i, j) at [j * 32 + i]
        double la[2][4];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
          for (int v = 0; v < 4; ++v) la[kb][v] = Li[(16 * kb + 4 * v + kl) * 32 + 16 * jb + li];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
          d4 nw = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int kb = 0; kb < 2; ++kb) {
            if (kb > jb) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v)
              nw = __builtin_amdgcn_mfma_f64_16x16x4f64(la[kb][v], Xs[(16 * kb + 4 * v + kl) * LDX + 16 * rb + li], nw,
                                                        0, 0, 0);
          }
          acc[rb][t] = nw;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int lc = 16 * jb + kl + 4 * v, row = 16 * rb + li;
            Xn[lc * LDX + row] = nw[v];
            xg[(size_t)(c0 + lc) * b + row] = nw[v];
            if (prec == PREC_FP32)
              gp(reinterpret_cast<float*>(low))[(size_t)(c0 + lc) * b + r0 + row] = (float)nw[v];
            else if (prec == PREC_BF16)
              gp(reinterpret_cast<uint16_t*>(low))[(size_t)(r0 + row) * b + c0 + lc] = to_bf16(nw[v]);
          }
        }
      }
    }
    __syncthreads();
    // (3) later blocks lose X_c L(j, c)^T
#pragma unroll
    for (int t = 0; t < NCB; ++t) {
      const int cb = wave + 4 * t;
      if (cb < ncb && cb >= cblk + 2) {
        double lf[8];
#pragma unroll
        for (int s4 = 0; s4 < 8; ++s4) lf[s4] = -lg[(size_t)(c0 + 4 * s4 + kl) * b + 16 * cb + li];
#pragma unroll
        for (int s4 = 0; s4 < 8; ++s4)
#pragma unroll
          for (int rb = 0; rb < 2; ++rb)
            acc[rb][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(lf[s4], Xn[(4 * s4 + kl) * LDX + 16 * rb + li],
                                                              acc[rb][t], 0, 0, 0);
      }
    }
  }
}

__device__ __noinline__ void trsm_part(double* __restrict__ x, const double* __restrict__ l, const double* __restrict__ dinv,
                          int b, int r0, void* __restrict__ low, int prec, double* __restrict__ lds, int k0 = 0) {
  if (b > 256)
    trsm_strip32<8>(x, l, dinv, b, r0, low, prec, lds, k0);
  else if (b > 128)
    trsm_strip32<4>(x, l, dinv, b, r0, low, prec, lds, k0);
  else if (b > 64)
    trsm_strip32<2>(x, l, dinv, b, r0, low, prec, lds, k0);
  else
    trsm_strip32<1>(x, l, dinv, b, r0, low, prec, lds, k0);
}

// Inverses of the 32x32 diagonal blocks of an already factored diagonal tile (one block
// per wave), for callers that run a TRSM or solve task on a factor they supplied.
__device__ void tile_inverses(const double* __restrict__ l, int b, double* __restrict__ dinv, double* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* D = lds + wave * 2048;
  double* Z = D + 1024;
  for (int c0 = 32 * wave; c0 < b; c0 += 32 * (NT / 64)) {
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int e = lane + 64 * t, r = e & 31, j = e >> 5;
      D[e] = r >= j ? l[(size_t)(c0 + j) * b + c0 + r] : 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    inverse32(D, Z);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int t = 0; t < 16; ++t) dinv[(size_t)c0 * 32 + lane + 64 * t] = Z[lane + 64 * t];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// ---------------------------------------------------------------------------------------
// Solve tasks on the right-hand side y (column-major, ld = n_pad), columns [q0, q0+nq).
// ---------------------------------------------------------------------------------------

// In-place block substitution (when no inverse of the diagonal tile was made): forward
// substitution of one diagonal tile for up to 8 right-hand sides: y_k <- L_kk^{-1}
// y_k, block by block (32 rows) with the inverted 32x32 diagonal blocks: y_blk <- Li y_blk,
// then the rows below lose L(rows, blk) y_blk.  The whole block of right-hand sides stays in
// LDS; thread t owns rows t and t + 256 of the trailing update, whose L strip for the next
// block is loaded into registers while the current block is solved, and the next block
// inverse is loaded into the other half of a double buffer.  Only the block-inverse
// products change the arithmetic order relative to a substitution.
__device__ void ftrsm_sub_part(const double* __restrict__ l, const double* __restrict__ dinv, int b,
                           double* __restrict__ y, int64_t ldy, int q0, int nq, double* __restrict__ lds, int na) {
  const int tid = threadIdx.x;
  LDSAS double* ys = lp(lds);            // [8][b] right-hand sides
  LDSAS double* Lb = lp(lds) + 8 * 512;  // two 32x32 block inverses
  LDSAS double* yb = Lb + 2048;  // [8][32] the block just solved
  const int q = tid >> 5, r = tid & 31;
  for (int e = tid; e < 8 * b; e += NT) {
    const int qq = e / b, m = e % b;
    ys[e] = qq < nq && m < na ? y[(size_t)(q0 + qq) * ldy + m] : 0.0;
  }
  for (int e = tid; e < 1024; e += NT) Lb[e] = dinv[e];
  double lv[2][32];
  auto load_strip = [&](int c0) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int row = tid + NT * j;
      if (row >= c0 + 32 && row < na) {
#pragma unroll
        for (int c = 0; c < 32; ++c) lv[j][c] = l[(size_t)(c0 + c) * b + row];
      }
    }
  };
  load_strip(0);
  int buf = 0;
  for (int c0 = 0; c0 < na; c0 += 32) {
    __syncthreads();  // block c0 of ys and the inverse in Lb[buf] are ready
    if (c0 + 32 < na)
      for (int e = tid; e < 1024; e += NT) Lb[(buf ^ 1) * 1024 + e] = dinv[(size_t)(c0 + 32) * 32 + e];
    const LDSAS double* Li = Lb + buf * 1024;
    if (q < nq) {
      double sacc = 0.0;
      for (int c = 0; c <= r; ++c) sacc += Li[c * 32 + r] * ys[q * b + c0 + c];
      yb[q * 32 + r] = sacc;
    }
    __syncthreads();
    if (q < nq) ys[q * b + c0 + r] = yb[q * 32 + r];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int row = tid + NT * j;
      if (row >= c0 + 32 && row < na) {
        double acc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = 0.0;
#pragma unroll
        for (int c = 0; c < 32; ++c)
#pragma unroll
          for (int u = 0; u < 8; ++u) acc[u] += lv[j][c] * yb[u * 32 + c];
        for (int u = 0; u < nq; ++u) ys[u * b + row] -= acc[u];
      }
    }
    if (c0 + 32 < na) load_strip(c0 + 32);
    buf ^= 1;
  }
  __syncthreads();
  for (int e = tid; e < nq * b; e += NT) {
    const int qq = e / b, m = e % b;
    if (m < na) y[(size_t)(q0 + qq) * ldy + m] = ys[e];
  }
}

// Backward: y_k <- L_kk^{-T} y_k, blocks from the last one down: x_blk = Li^T y_blk, then
// the rows above lose L(blk, rows)^T x_blk.  Row t's strip L(c0 .. c0+31, t) is contiguous
// (column t of the tile); otherwise as the forward substitution (the padding blocks are
// zero and contribute nothing, so starting at the block below na changes no bit).
__device__ void btrsm_sub_part(const double* __restrict__ l, const double* __restrict__ dinv, int b,
                           double* __restrict__ y, int64_t ldy, int q0, int nq, double* __restrict__ lds, int na) {
  const int tid = threadIdx.x;
  LDSAS double* ys = lp(lds);
  LDSAS double* Lb = lp(lds) + 8 * 512;
  LDSAS double* yb = Lb + 2048;
  const int q = tid >> 5, r = tid & 31;
  for (int e = tid; e < 8 * b; e += NT) {
    const int qq = e / b, m = e % b;
    ys[e] = qq < nq && m < na ? y[(size_t)(q0 + qq) * ldy + m] : 0.0;
  }
  for (int e = tid; e < 1024; e += NT) Lb[e] = dinv[(size_t)(na - 32) * 32 + e];
  double lv[2][32];
  auto load_strip = [&](int c0) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int row = tid + NT * j;
      if (row < c0) {
        const double2* src = reinterpret_cast<const double2*>(l + (size_t)row * b + c0);
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const double2 v = src[c];
          lv[j][2 * c] = v.x;
          lv[j][2 * c + 1] = v.y;
        }
      }
    }
  };
  load_strip(na - 32);
  int buf = 0;
  for (int c0 = na - 32; c0 >= 0; c0 -= 32) {
    __syncthreads();
    if (c0 > 0)
      for (int e = tid; e < 1024; e += NT) Lb[(buf ^ 1) * 1024 + e] = dinv[(size_t)(c0 - 32) * 32 + e];
    const LDSAS double* Li = Lb + buf * 1024;
    if (q < nq) {
      double sacc = 0.0;
      for (int c = r; c < 32; ++c) sacc += Li[r * 32 + c] * ys[q * b + c0 + c];  // Li(c, r)
      yb[q * 32 + r] = sacc;
    }
    __syncthreads();
    if (q < nq) ys[q * b + c0 + r] = yb[q * 32 + r];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int row = tid + NT * j;
      if (row < c0) {
        double acc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = 0.0;
#pragma unroll
        for (int c = 0; c < 32; ++c)
#pragma unroll
          for (int u = 0; u < 8; ++u) acc[u] += lv[j][c] * yb[u * 32 + c];
        for (int u = 0; u < nq; ++u) ys[u * b + row] -= acc[u];
      }
    }
    if (c0 > 0) load_strip(c0 - 32);
    buf ^= 1;
  }
  __syncthreads();
  for (int e = tid; e < nq * b; e += NT) {
    const int qq = e / b, m = e % b;
    if (m < na) y[(size_t)(q0 + qq) * ldy + m] = ys[e];
  }
}

// ---------------------------------------------------------------------------------------
// Solve parts (few right-hand sides): R output rows per part (64, or 32 for 32-wide
// tiles).  For rows r in [r0, r0+R) and right-hand sides q < nq:
//   s(r, q) = sum over k in [kb, ke) of A(r, k) ys[q][k],
// with A(r, k) at A[k lda + r] (COLS: the rows of a column are contiguous) or at
// A[r lda + k] (ROWS: a row is contiguous); kb, ke, r0 and lda are multiples of 4.  Every
// load is 32 bytes (4 rows of a column, or 4 entries of a row), so each thread has only
// R b / 1024 loads, all independent and issued together: the part costs about one
// memory round trip instead of a chain of them.  COLS: thread t takes rows 4 (t % (R/4))
// .. +3 and every G-th k from t / (R/4) (G = 1024 / R groups); ROWS: row t / (256/R) and
// every 4-entry chunk 4 (t % (256/R)) + 1024/R * s.  The partial sums of a row are added
// through LDS in a fixed order.  ys: 8 columns of stride ysd in LDS.  Leaves s(r0 + r, q)
// in sums[q R + r] (LDS) for every thread to read after the closing barrier.
// ---------------------------------------------------------------------------------------
template <int R, bool ROWS>
__device__ void skinny_rows(const double* __restrict__ A, int lda, int r0, int kb, int ke,
                            const LDSAS double* ys, int ysd, int nq, LDSAS double* partial, LDSAS double* sums) {
  constexpr int G = ROWS ? NT / R : NT / (R / 4);  // partial sums per row
  const int tid = threadIdx.x;
  double acc[4][8];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[v][q] = 0.0;
  int g;
  if (ROWS) {
    const int i = tid / G;
    g = tid % G;
    const double* row = A + (size_t)(r0 + i) * lda;
    // acc[v][q]: the four entries of a chunk kept apart, summed at the end (fixed order)
    if (nq == 1) {
#pragma unroll 8
      for (int k = kb + 4 * g; k < ke; k += 4 * G) {
        const double4 a = *reinterpret_cast<const double4*>(row + k);
        acc[0][0] += a.x * ys[k];
        acc[1][0] += a.y * ys[k + 1];
        acc[2][0] += a.z * ys[k + 2];
        acc[3][0] += a.w * ys[k + 3];
      }
    } else {
#pragma unroll 2
      for (int k = kb + 4 * g; k < ke; k += 4 * G) {
        const double4 a = *reinterpret_cast<const double4*>(row + k);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          acc[0][q] += a.x * ys[q * ysd + k];
          acc[1][q] += a.y * ys[q * ysd + k + 1];
          acc[2][q] += a.z * ys[q * ysd + k + 2];
          acc[3][q] += a.w * ys[q * ysd + k + 3];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[0][q] = (acc[0][q] + acc[1][q]) + (acc[2][q] + acc[3][q]);
  } else {
    const int i4 = tid % (R / 4);
    g = tid / (R / 4);
    const double* col = A + r0 + 4 * i4;
    if (nq == 1) {
#pragma unroll 8
      for (int k = kb + g; k < ke; k += G) {
        const double4 a = *reinterpret_cast<const double4*>(col + (size_t)k * lda);
        const double y = ys[k];
        acc[0][0] += a.x * y;
        acc[1][0] += a.y * y;
        acc[2][0] += a.z * y;
        acc[3][0] += a.w * y;
      }
    } else {
#pragma unroll 2
      for (int k = kb + g; k < ke; k += G) {
        const double4 a = *reinterpret_cast<const double4*>(col + (size_t)k * lda);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const double y = ys[q * ysd + k];
          acc[0][q] += a.x * y;
          acc[1][q] += a.y * y;
          acc[2][q] += a.z * y;
          acc[3][q] += a.w * y;
        }
      }
    }
  }
  __syncthreads();  // the caller's earlier use of `partial` is over
  if (ROWS) {
    const int i = tid / G;
#pragma unroll
    for (int q = 0; q < 8; ++q) partial[(q * G + g) * R + i] = acc[0][q];
  } else {
    const int i4 = tid % (R / 4);
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) partial[(q * G + g) * R + 4 * i4 + v] = acc[v][q];
  }
  __syncthreads();
  for (int e = tid; e < R * nq; e += NT) {
    const int ri = e % R, q = e / R;
    double sum = 0.0;
#pragma unroll
    for (int gg = 0; gg < G; ++gg) sum += partial[(q * G + gg) * R + ri];
    sums[e] = sum;
  }
  __syncthreads();
}

// Stages columns q0 .. q0+nq-1, entries [kb, ke), of a right-hand-side block into LDS
// (8 columns of stride b; the other entries are not read).
__device__ __forceinline__ void stage_rhs(const double* __restrict__ y, int64_t ldy, int q0, int nq, int b, int kb,
                                          int ke, LDSAS double* ys) {
  const int w = ke - kb;
  for (int e = threadIdx.x; e < 8 * w; e += NT) {
    const int q = e / w, m = kb + e % w;
    ys[q * b + m] = q < nq ? y[(size_t)(q0 + q) * ldy + m] : 0.0;
  }
  __syncthreads();
}

// ys at lds[0, 4096), the partial sums at [4096, 12288), the sums at [12288, 12800).
template <bool ROWS>
__device__ __forceinline__ void skinny(int rows, const double* A, int lda, int r0, int kb, int ke,
                                       const LDSAS double* ys, int ysd, int nq, LDSAS double* partial,
                                       LDSAS double* sums) {
  if (rows == 64)
    skinny_rows<64, ROWS>(A, lda, r0, kb, ke, ys, ysd, nq, partial, sums);
  else
    skinny_rows<32, ROWS>(A, lda, r0, kb, ke, ys, ysd, nq, partial, sums);
}

// Diagonal solves with M_k = L_kk^{-T} (column-major b x b; upper triangular: made by the
// inversion task, exact zeros below its diagonal), rows [r0, r0+rows) for one group of up
// to 8 right-hand sides, from yin to yout (another buffer, so the strips of a block run as
// separate parts): forward y(r) = sum over c <= r of M(c, r) b(c) (column r of M, read as
// row r of M^T, contiguous); backward x(r) = sum over c >= r of M(r, c) y(c).
__device__ void ftrsm_rows(const double* __restrict__ M, int b, const double* __restrict__ yin,
                           double* __restrict__ yout, int64_t ldy, int q0, int nq, int r0, int rows,
                           double* __restrict__ lds) {
  LDSAS double* ys = lp(lds);
  LDSAS double* partial = ys + 8 * 512;
  LDSAS double* sums = partial + 8 * 1024;
  stage_rhs(yin, ldy, q0, nq, b, 0, r0 + rows, ys);
  skinny<true>(rows, M, b, r0, 0, r0 + rows, ys, b, nq, partial, sums);
  for (int e = threadIdx.x; e < rows * nq; e += NT) yout[(size_t)(q0 + e / rows) * ldy + r0 + e % rows] = sums[e];
}

__device__ void btrsm_rows(const double* __restrict__ M, int b, const double* __restrict__ yin,
                           double* __restrict__ yout, int64_t ldy, int q0, int nq, int r0, int rows,
                           double* __restrict__ lds) {
  LDSAS double* ys = lp(lds);
  LDSAS double* partial = ys + 8 * 512;
  LDSAS double* sums = partial + 8 * 1024;
  stage_rhs(yin, ldy, q0, nq, b, r0, b, ys);
  skinny<false>(rows, M, b, r0, r0, b, ys, b, nq, partial, sums);
  for (int e = threadIdx.x; e < rows * nq; e += NT) yout[(size_t)(q0 + e / rows) * ldy + r0 + e % rows] = sums[e];
}

// Off-diagonal updates, rows [r0, r0+rows) of block i, every right-hand side (8 at a
// time): forward y_i -= L_ik y_k (tile (i,k), rows of a column contiguous); backward
// y_i -= L_ki^T y_k (tile (k,i): row r of L_ki^T is column r of the tile, contiguous).
// Each row's old value is read after the sums, by the thread that writes it.
template <bool BACKWARD>
__device__ void update_rows(const double* __restrict__ l, int b, double* __restrict__ yi,
                            const double* __restrict__ yk, int64_t ldy, int nrhs, int r0, int rows,
                            double* __restrict__ lds) {
  LDSAS double* ys = lp(lds);
  LDSAS double* partial = ys + 8 * 512;
  LDSAS double* sums = partial + 8 * 1024;
  for (int q0 = 0; q0 < nrhs; q0 += 8) {
    const int nq = (nrhs - q0) < 8 ? (nrhs - q0) : 8;
    // (the previous group's reads of ys and sums ended before its closing barrier)
    stage_rhs(yk, ldy, q0, nq, b, 0, b, ys);
    skinny<BACKWARD>(rows, l, b, r0, 0, b, ys, b, nq, partial, sums);
    for (int e = threadIdx.x; e < rows * nq; e += NT) {
      double* p = yi + (size_t)(q0 + e / rows) * ldy + r0 + e % rows;
      *p = *p - sums[e];
    }
    __syncthreads();  // sums read before the next group overwrites ys and sums
  }
}

// Sub-block (si, sj) of size S x S of tile (ti, tj); s: 64 x 65 doubles of LDS.
// Every thread's S*S/NT elements are loaded (all loads issued together) before any is
// stored to LDS, and read back from LDS before any global store: one memory round trip
// each way per sub-block.
template <int S>
__device__ void pack_block_s(const double* __restrict__ A, int64_t lda, int64_t n, const DevMat& m, int ti, int tj,
                             int si, int sj, double* __restrict__ s) {
  constexpr int PER = S * S / NT;
  const int b = m.b;
  const int64_t R0 = (int64_t)ti * b + si * S, C0 = (int64_t)tj * b + sj * S;
  LDSAS double* sl = lp(s);
  const GLOBAL double* Ag = gp(A);
  double v[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT, rr = e / S, cc = e % S;  // cc fastest: row-major reads
    const int64_t R = R0 + rr, C = C0 + cc;
    v[i] = (R < n && C < n) ? (R >= C ? Ag[R * lda + C] : 0.0) : (R == C ? 1.0 : 0.0);
  }
  if (m.dscale) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + i * NT, rr = e / S, cc = e % S;
      const int64_t R = R0 + rr, C = C0 + cc;
      if (R < n && C < n) {
        v[i] = v[i] * m.dscale[R] * m.dscale[C];
        if (R == C) v[i] += m.shift;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    sl[(e / S) * 65 + e % S] = v[i];
  }
  __syncthreads();
  GLOBAL double* T = gp(tile_ptr(m, ti, tj));
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT, cc = e / S, rr = e % S;  // rr fastest: column-major writes
    v[i] = sl[rr * 65 + cc];
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT, cc = e / S, rr = e % S;
    T[(size_t)(sj * S + cc) * b + si * S + rr] = v[i];
  }
  __syncthreads();
}

// A whole tile (ti, tj) by one workgroup, as pack_block_s<64> does each 64x64 block, with
// the next block's loads issued before the current one goes through LDS, so about two
// blocks of reads are in flight instead of one.  live_rows > 0: only the blocks on or
// below the diagonal whose rows start below live_rows are packed (the others are never
// read by the launch).
__device__ __noinline__ void pack_tile64(const double* __restrict__ A, int64_t lda, int64_t n, const DevMat& m,
                                         int ti, int tj, double* __restrict__ s, int live_rows = 0) {
  constexpr int S = 64, PER = S * S / NT;
  const int b = m.b, per = b / S, nblk = per * per;
  auto live = [&](int q) {
    const int si = q / per, sj = q % per;
    return live_rows <= 0 || (sj <= si && si * S < live_rows);
  };
  auto next_live = [&](int q) {
    do ++q;
    while (q < nblk && !live(q));
    return q;
  };
  LDSAS double* sl = lp(s);
  const GLOBAL double* Ag = gp(A);
  GLOBAL double* T = gp(tile_ptr(m, ti, tj));
  double cur[PER], nxt[PER];
  auto load = [&](int q, double (&v)[PER]) {
    const int64_t R0 = (int64_t)ti * b + (q / per) * S, C0 = (int64_t)tj * b + (q % per) * S;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + i * NT, rr = e / S, cc = e % S;  // cc fastest: row-major reads
      const int64_t R = R0 + rr, C = C0 + cc;
      v[i] = (R < n && C < n) ? (R >= C ? Ag[R * lda + C] : 0.0) : (R == C ? 1.0 : 0.0);
    }
  };
  int q = live(0) ? 0 : next_live(0);
  if (q < nblk) load(q, cur);
  while (q < nblk) {
    const int qn = next_live(q);
    if (qn < nblk) load(qn, nxt);
    const int si = q / per, sj = q % per;
    if (m.dscale) {
      const int64_t R0 = (int64_t)ti * b + si * S, C0 = (int64_t)tj * b + sj * S;
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = threadIdx.x + i * NT, rr = e / S, cc = e % S;
        const int64_t R = R0 + rr, C = C0 + cc;
        if (R < n && C < n) {
          cur[i] = cur[i] * m.dscale[R] * m.dscale[C];
          if (R == C) cur[i] += m.shift;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + i * NT;
      sl[(e / S) * 65 + e % S] = cur[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + i * NT, cc = e / S, rr = e % S;  // rr fastest: column-major writes
      cur[i] = sl[rr * 65 + cc];
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + i * NT, cc = e / S, rr = e % S;
      T[(size_t)(sj * S + cc) * b + si * S + rr] = cur[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) cur[i] = nxt[i];
    q = qn;
  }
}

__device__ void pack_block(const double* __restrict__ A, int64_t lda, int64_t n, const DevMat& m, int ti, int tj,
                           int si, int sj, int S, double* __restrict__ s) {
  if (S == 64) {
    pack_block_s<64>(A, lda, n, m, ti, tj, si, sj, s);
    return;
  }
  if (S == 32) {
    pack_block_s<32>(A, lda, n, m, ti, tj, si, sj, s);
    return;
  }
  const int b = m.b;
  const int64_t R0 = (int64_t)ti * b + si * S, C0 = (int64_t)tj * b + sj * S;
  for (int e = threadIdx.x; e < S * S; e += NT) {
    const int rr = e / S, cc = e % S;  // cc fastest: row-major reads
    const int64_t R = R0 + rr, C = C0 + cc;
    double v;
    if (R < n && C < n) {
      v = (R >= C) ? A[R * lda + C] : 0.0;
      if (m.dscale) {
        v = v * m.dscale[R] * m.dscale[C];
        if (R == C) v += m.shift;
      }
    } else {
      v = (R == C) ? 1.0 : 0.0;
    }
    s[rr * 65 + cc] = v;
  }
  __syncthreads();
  double* T = tile_ptr(m, ti, tj);
  for (int e = threadIdx.x; e < S * S; e += NT) {
    const int cc = e / S, rr = e % S;  // rr fastest: column-major writes
    T[(size_t)(sj * S + cc) * b + si * S + rr] = s[rr * 65 + cc];
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------------------
// Part dispatch.
// ---------------------------------------------------------------------------------------
__device__ __attribute__((noinline)) void run_part_chol(const SchedArgs& a, uint32_t task, uint32_t part,
                                                        double* lds) {
  const TaskDesc d = a.tasks[task];
  const DevMat& m = a.mats[d.mat];
  // a failed pivot earlier in this matrix: its remaining tasks drain without computing
  if (__hip_atomic_load(m.info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != INT_MAX) return;
  const int b = m.b;
  switch (d.type) {
    case SPX_T_POTRF: {
      // pad = step | (steps << 8) when the factorization is split into steps
      const int steps = d.pad >> 8;
      const int na = tile_active(m, d.k);
      const int bad = steps > 1 ? potrf_step_part(tile_ptr(m, d.k, d.k), b, dinv_ptr(m, d.k), d.pad & 0xff, (int)part, lds, na)
                                : potrf_tile(tile_ptr(m, d.k, d.k), b, dinv_ptr(m, d.k), lds, na);
      if (bad && threadIdx.x == 0)
        __hip_atomic_fetch_min(m.info, d.k * b + bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    case SPX_T_TRSM: {
      const int R = m.trsm_rows;
      const size_t off = ((size_t)d.i * (d.i + 1) / 2 + d.k) * (size_t)b * b;
      void* low = m.prec == PREC_FP32   ? (void*)(reinterpret_cast<float*>(m.low) + off)
                  : m.prec == PREC_BF16 ? (void*)(reinterpret_cast<uint16_t*>(m.low) + off)
                                        : nullptr;
      const int r0 = (int)part * R;
      if (r0 >= tile_active(m, d.i)) {  // a strip of zero padding rows: X stays zero
        if (low) {  // its low-precision copy is read by the updates: clear it (the FP32
                    // copy is column-major, the BF16 copy row-major, as the TRSM writes them)
          for (int e = threadIdx.x; e < R * b; e += NT) {
            if (m.prec == PREC_FP32)
              reinterpret_cast<float*>(low)[(size_t)(e / R) * b + r0 + e % R] = 0.0f;
            else
              reinterpret_cast<uint16_t*>(low)[(size_t)(r0 + e / b) * b + e % b] = 0;
          }
        }
        break;
      }
      trsm_part(tile_ptr(m, d.i, d.k), tile_ptr(m, d.k, d.k), dinv_ptr(m, d.k), b, r0, low, m.prec, lds);
      break;
    }
    case SPX_T_SYRK:
    case SPX_T_GEMM: {
      // part -> 128x128 sub-block (I, J) of the output tile (64x64 for the SYRK that the
      // next diagonal factorization waits on); SYRK: lower blocks only
      const int sbase = (d.type == SPX_T_SYRK && d.pad) ? 64 : 128;
      const int sb = b < sbase ? b : sbase, ns = b / sb;
      int I, J;
      if (d.type == SPX_T_SYRK) {
        I = 0;
        while ((I + 1) * (I + 2) / 2 <= (int)part) ++I;
        J = part - I * (I + 1) / 2;
      } else {
        I = part % ns;
        J = part / ns;
      }
      // a sub-block of the last tile row's padding rows or columns: its entries stay
      if (I * sb >= tile_active(m, d.i) || J * sb >= tile_active(m, d.j)) break;
      double* C = tile_ptr(m, d.i, d.j) + (size_t)J * sb * b + I * sb;
      const bool lower = d.type == SPX_T_SYRK && I == J;
      const size_t oi = ((size_t)d.i * (d.i + 1) / 2 + d.k) * (size_t)b * b;
      const size_t oj = ((size_t)d.j * (d.j + 1) / 2 + d.k) * (size_t)b * b;
      if (m.prec == PREC_FP32) {
        const float* lf = reinterpret_cast<const float*>(m.low);
        const float* Ai = lf + oi + I * sb;
        const float* Bj = lf + oj + J * sb;
        if (sb > 64) gemm_nt_f32<64>(C, b, Ai, b, Bj, b, sb, sb, b, lower, lds);
        else if (sb > 32) gemm_nt_f32<32>(C, b, Ai, b, Bj, b, sb, sb, b, lower, lds);
        else gemm_nt_f32<16>(C, b, Ai, b, Bj, b, sb, sb, b, lower, lds);
      } else if (m.prec == PREC_BF16) {
        const uint16_t* lh = reinterpret_cast<const uint16_t*>(m.low);
        const uint16_t* Ai = lh + oi + (size_t)I * sb * b;
        const uint16_t* Bj = lh + oj + (size_t)J * sb * b;
        if (sb > 64) gemm_nt_bf16<64>(C, b, Ai, b, Bj, b, sb, sb, b, lower, lds);
        else if (sb > 32) gemm_nt_bf16<32>(C, b, Ai, b, Bj, b, sb, sb, b, lower, lds);
        else gemm_nt_bf16<16>(C, b, Ai, b, Bj, b, sb, sb, b, lower, lds);
      } else {
        const double* Ai = tile_ptr(m, d.i, d.k) + I * sb;
        const double* Bj = tile_ptr(m, d.j, d.k) + J * sb;
        gemm_nt_any(C, b, Ai, b, Bj, b, sb, sb, b, lower, lds);
      }
      break;
    }
    case SPX_T_FTRSM:
    case SPX_T_BTRSM: {
      if (!d.pad) {  // in-place block substitution, one part per group of 8 right-hand sides
        const int q0 = part * 8, nq = (m.nrhs - q0) < 8 ? (m.nrhs - q0) : 8;
        if (d.type == SPX_T_FTRSM)
          ftrsm_sub_part(tile_ptr(m, d.k, d.k), dinv_ptr(m, d.k), b, m.rhs + (size_t)d.k * b, m.n_pad, q0, nq, lds,
                         tile_active(m, d.k));
        else
          btrsm_sub_part(tile_ptr(m, d.k, d.k), dinv_ptr(m, d.k), b, m.rhs + (size_t)d.k * b, m.n_pad, q0, nq, lds,
                         tile_active(m, d.k));
        break;
      }
      // with M_k: part -> (group of 8 right-hand sides, strip of 64 rows)
      const int rows = b < 64 ? b : 64, nrp = b / rows;
      const int q0 = ((int)part / nrp) * 8, nq = (m.nrhs - q0) < 8 ? (m.nrhs - q0) : 8;
      const int r0 = ((int)part % nrp) * rows;
      const double* Mk = m.minv + (size_t)d.k * b * b;
      if (d.type == SPX_T_FTRSM)
        ftrsm_rows(Mk, b, m.rhs + (size_t)d.k * b, m.rhs2 + (size_t)d.k * b, m.n_pad, q0, nq, r0, rows, lds);
      else
        btrsm_rows(Mk, b, m.rhs2 + (size_t)d.k * b, m.rhs + (size_t)d.k * b, m.n_pad, q0, nq, r0, rows, lds);
      break;
    }
    case SPX_T_INV: {
      // rows [r0, r0 + R) of M_k = I L_kk^{-T}: identity rows, then the TRSM strip kernel
      const int R = m.trsm_rows, r0 = part * R;
      double* x = m.minv + (size_t)d.k * b * b;
      for (int e = threadIdx.x; e < R * b; e += NT) {
        const int c = e / R, r = e % R;
        x[(size_t)c * b + r0 + r] = (r0 + r == c) ? 1.0 : 0.0;
      }
      __syncthreads();
      trsm_part(x, tile_ptr(m, d.k, d.k), dinv_ptr(m, d.k), b, r0, nullptr, PREC_FP64, lds, r0 & ~31);
      break;
    }
    case SPX_T_FGEMM: {  // one strip of 64 rows per part
      const int rows = b < 64 ? b : 64;
      update_rows<false>(tile_ptr(m, d.i, d.k), b, m.rhs + (size_t)d.i * b,
                         (d.pad ? m.rhs2 : m.rhs) + (size_t)d.k * b, m.n_pad, m.nrhs, (int)part * rows, rows, lds);
      break;
    }
    case SPX_T_BGEMM: {
      // task (i, k): y_i -= L_ki^T y_k; the tile is (k, i) with k = d.j
      const int rows = b < 64 ? b : 64;
      update_rows<true>(tile_ptr(m, d.j, d.i), b, (d.pad ? m.rhs2 : m.rhs) + (size_t)d.i * b,
                        m.rhs + (size_t)d.j * b, m.n_pad, m.nrhs, (int)part * rows, rows, lds);
      break;
    }
    case SPX_T_LOAD: {
      // one part per lower tile (per tile row if the tiles outnumber the part index), then
      // one for the right-hand sides
      const int ntiles = m.nt * (m.nt + 1) / 2;
      const bool per_tile = ntiles <= kLoadTileParts;
      const int ndata = per_tile ? ntiles : m.nt;
      if (d.j == 0 && (int)part < ndata) {
        const int S = b < 64 ? b : 64, per = b / S;
        int ti = (int)part, tj0 = 0, tj1 = (int)part;  // a tile row
        if (per_tile) {
          ti = (int)((sqrt(8.0 * part + 1.0) - 1.0) * 0.5);
          while (ti * (ti + 1) / 2 > (int)part) --ti;
          while ((ti + 1) * (ti + 2) / 2 <= (int)part) ++ti;
          tj0 = tj1 = (int)part - ti * (ti + 1) / 2;
        }
        for (int tj = tj0; tj <= tj1; ++tj) {
          if (S == 64) pack_tile64(m.A, m.lda, m.n, m, ti, tj, lds, m.load_live ? tile_active(m, ti) : 0);
          else
            for (int q = 0; q < per * per; ++q) pack_block(m.A, m.lda, m.n, m, ti, tj, q / per, q % per, S, lds);
        }
      } else {
        const int64_t total = m.n_pad * m.nrhs;
        for (int64_t e = threadIdx.x; e < total; e += NT) {
          const int64_t q = e / m.n_pad, r = e % m.n_pad;
          m.rhs[e] = r < m.n ? m.B[r * m.ldb + q] : 0.0;
        }
      }
      break;
    }
    case SPX_T_STORE: {
      const int64_t total = (int64_t)m.n * m.nrhs;
      for (int64_t e = threadIdx.x; e < total; e += NT) {
        const int64_t r = e / m.nrhs, q = e % m.nrhs;
        if (m.store_acc)
          m.X[r * m.ldx + q] += m.rhs[q * m.n_pad + r];
        else
          m.X[r * m.ldx + q] = m.rhs[q * m.n_pad + r];
      }
      break;
    }
    default:
      break;
  }
}

// The tiled product's task, C_ij += A_ik B_kj (the GEMM application): part -> 128x128
// sub-block (I, J) of C_ij; the B operand is the tile (j, k) of B^T, so the transposed-B
// update applies with the sign turned.  Every block is full, so the guard-free loads.
__device__ __attribute__((noinline)) void run_part_gemm(const SchedArgs& a, uint32_t task, uint32_t part,
                                                        double* lds) {
  const TaskDesc d = a.tasks[task];
  const DevMat& m = a.mats[d.mat];
  const int b = m.b;
  const int sb = b < 128 ? b : 128, ns = b / sb;
  const int I = part % ns, J = part / ns;
  const size_t bb = (size_t)b * b;
  double* C = m.tiles + ((size_t)d.i * m.nt + d.j) * bb + (size_t)J * sb * b + I * sb;
  const double* Ai = m.ga + ((size_t)d.i * m.nt + d.k) * bb + I * sb;
  const double* Bj = m.gbt + ((size_t)d.j * m.nt + d.k) * bb + J * sb;
  if (sb > 64)
    gemm_nt_f64<64, true>(C, b, Ai, b, Bj, b, sb, sb, b, false, lds, -1.0);
  else if (sb > 32)
    gemm_nt_f64<32, true>(C, b, Ai, b, Bj, b, sb, sb, b, false, lds, -1.0);
  else
    gemm_nt_f64<16, true>(C, b, Ai, b, Bj, b, sb, sb, b, false, lds, -1.0);
}

// The empty task of the overhead study: one lane watches the clock for the task's
// duration, the other lanes wait at the barrier that ends every part.
__device__ __attribute__((noinline)) void run_part_spin(const SchedArgs& a, uint32_t task, uint32_t,
                                                        double*) {
  const DevMat& m = a.mats[a.tasks[task].mat];
  if (threadIdx.x == 0) {
    const u64 t0 = now_ticks();
    while (now_ticks() - t0 < m.spin_ticks) __builtin_amdgcn_s_sleep(1);
  }
}

// Task families: a launch runs the scheduler instantiated for the task types its graph
// can hold, so each instantiation holds (and allocates registers for) only those tile
// kernels.  The task bodies stay out of line and the scheduler's queue operations inline,
// the code layout under which the Cholesky kernel compiles without VGPR spills (inlining
// the task bodies into the loop, or adding the tiled product to them, made the compiler
// spill 24-113 VGPRs).
template <int FAM>
__device__ __forceinline__ void run_part(const SchedArgs& a, uint32_t task, uint32_t part, double* lds) {
  if constexpr (FAM == FAM_CHOL)
    run_part_chol(a, task, part, lds);
  else if constexpr (FAM == FAM_GEMM)
    run_part_gemm(a, task, part, lds);
  else
    run_part_spin(a, task, part, lds);
}

// ---------------------------------------------------------------------------------------
// The persistent scheduler kernel.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ u64* ctr_queue(const SchedArgs& a, int l, int s) {
  return reinterpret_cast<u64*>(a.counters + ctr_queue_idx(l * a.nshards + s));
}
__device__ __forceinline__ uint32_t* ctr_status(const SchedArgs& a) { return a.counters + kStatusIdx; }
__device__ __forceinline__ u64* queue_of(const SchedArgs& a, int l, int s) {
  return a.queue + (size_t)a.qbase[l] * kShards + (size_t)s * a.qcap[l];
}

// Memory ordering.  All counter and queue updates are relaxed; visibility of tile data
// comes from agent-scope fences, which on this chip write back (release) or invalidate
// (acquire) the L2 of the XCD that runs them.  A release costs microseconds and the
// write-backs of one XCD's L2 do not overlap, so a release per finished part would queue
// every workgroup behind its XCD's other 31; instead each XCD releases in rounds:
//   * a finished claim appends its tasks to its XCD's ring (its stores are in that XCD's
//     L2: the barrier before waited for them) and tries the XCD's round lock;
//   * the lock holder reads the ring's tail, runs one release (which writes back every
//     part appended before that read, all of them in this L2), then decrements parts_left
//     for each of them and, for a task's last part, the successors' pending counters,
//     pushing the ready ones; it repeats while the ring grows, and after unlocking looks
//     once more, so an entry whose appender found the lock taken is never left behind;
//   * a popped part: the task's pending counter is read (0: every predecessor's last part
//     was written back before its decrement), then one acquire fence drops this XCD's
//     stale lines.
__device__ __forceinline__ void fence_rel() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void fence_acq() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ uint32_t sub_rlx(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_sub(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The XCD this wave runs on (hardware register; its low three bits number the XCDs).
__device__ __forceinline__ int xcd_id() {
  uint32_t v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return (int)(v & (kXcds - 1));
}

// Push task s (descriptor d) at shard home of its level: reserve slots, then fill them.
// In a launch that allows it, a task of at most a.spread_max (<= kSpreadMax) parts deals
// them over the shards, part p into shard (home + p % w) % S with w = min(nparts, S): the
// claims of its parts then go to w queue heads at once instead of one after another on a
// single head (the claims on one head serialise at a microsecond or more each, which
// spread the starts of a latency-bound substitution's eight-part tasks over up to 30 us).
// Larger tasks keep their parts together, where multi-part claims take them; the
// substitution tasks, latency-bound, spread up to twice as many (a diagonal solve of 9 to
// 16 right-hand sides has 16 parts).
constexpr uint32_t kSpreadMax = 8;
__device__ __forceinline__ void push_task(const SchedArgs& a, uint32_t s, const TaskDesc& d, int home) {
  const uint32_t S = (uint32_t)a.nshards, np = d.nparts;
  const bool subst = d.type >= SPX_T_FTRSM && d.type <= SPX_T_BGEMM;
  const uint32_t lim = subst ? 2u * a.spread_max : a.spread_max;
  const uint32_t w = np > 1u && np <= lim && np <= 2u * kSpreadMax ? (np < S ? np : S) : 1u;
  uint32_t slot[kShards];
#pragma unroll
  for (uint32_t k = 0; k < (uint32_t)kShards; ++k) {
    if (k < w) {
      uint32_t sh = (uint32_t)home + k;
      sh -= sh >= S ? S : 0u;
      const uint32_t cnt = (np - k + w - 1u) / w;  // parts k, k + w, ...
      slot[k] = (uint32_t)(__hip_atomic_fetch_add(ctr_queue(a, d.level, (int)sh), (u64)cnt << 32, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT) >> 32);
    }
  }
#pragma unroll
  for (uint32_t k = 0; k < (uint32_t)kShards; ++k) {
    if (k < w) {
      uint32_t sh = (uint32_t)home + k;
      sh -= sh >= S ? S : 0u;
      u64* q = queue_of(a, d.level, (int)sh) + slot[k];
      for (uint32_t p = k, e = 0; p < np; p += w, ++e)
        __hip_atomic_store(q + e, ((u64)s << 16) | p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (a.trace_push) a.trace_push[s] = now_ticks();
}
__device__ __forceinline__ void push_task(const SchedArgs& a, uint32_t s, int home) {
  push_task(a, s, a.tasks[s], home);
}

// pop, run by all 64 lanes of wave 0: lane i reads the head and tail of queue (level
// i / S, shard (home + i) % S) for the S shards in use, all in one round trip; the lowest
// lane with a non-empty queue (highest priority level, own shard first) claims slots with
// a compare-and-swap, retried in place with the head it returns.  It claims several parts
// at once while the queue is long (2 from 32 waiting, 4 from 128 on any level where the
// launch allows it, a.max_claim; from 64, 128 and 192 on the bulk levels, the lowest
// quarter): the compare-and-swaps on one shared
// head serialise at about one per microsecond, which with single claims left a tenth to
// a half of the workgroups idle while thousands of parts waited (N = 16384 factor: 43.5
// -> 40.1 ms), and each claim costs one release fence.
// Writes up to kClaim items to items[] (lane 0's copy) and returns their number (the same
// in every lane); *saw tells whether some queue looked non-empty and *taken is the number
// of parts taken from all queues so far (never more than the true count).
constexpr int kClaim = 4;
__device__ __forceinline__ int pop_wave(const SchedArgs& a, int home, bool* saw, uint32_t* taken, u64* items) {
  const int lane = threadIdx.x & 63, S = a.nshards;
  const bool valid = lane < a.nlev * S;
  const int l = lane / S, sh = (home + lane % S) % S;
  u64 ht = 0;
  if (valid) ht = __hip_atomic_load(ctr_queue(a, l, sh), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint32_t h = (uint32_t)ht, t = (uint32_t)(ht >> 32);
  uint32_t sum = h;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) sum += __shfl_xor(sum, off);
  *taken = sum;
  const unsigned long long mask = __ballot(valid && h < t);
  *saw = mask != 0ull;
  if (!mask) return 0;
  const int win = __ffsll((long long)mask) - 1;
  int k = 0;
  u64 it[kClaim];
#pragma unroll
  for (int i = 0; i < kClaim; ++i) it[i] = EMPTY;
  if (lane == win) {
    const bool bulk = a.nlev > 2 && l >= a.nlev - a.nlev / 4;
    for (;; h = (uint32_t)ht, t = (uint32_t)(ht >> 32)) {
      if (h >= t) break;
      const uint32_t avail = t - h;
      const uint32_t want = bulk ? (avail >= 192u ? 4u : avail >= 128u ? 3u : avail >= 64u ? 2u : 1u)
                                 : (a.max_claim < 2u ? 1u : avail >= 128u ? 4u : avail >= 32u ? 2u : 1u);
      // a push between the load and the swap changes the tail half and fails the swap:
      // retry with the word it returns
      if (__hip_atomic_compare_exchange_strong(ctr_queue(a, l, sh), &ht, ht + want, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        // the slots are reserved by running pushers: wait for the items to be written
        // (bounded by the spin limit: a slot still empty then ends the launch)
        const u64* q = queue_of(a, l, sh) + h;
        const u64 t0 = now_ticks();
        k = (int)want;
#pragma unroll
        for (int i = 0; i < kClaim; ++i) {
          if (i < (int)want) {
            u64 v;
            while ((v = __hip_atomic_load(q + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == EMPTY) {
              if (now_ticks() - t0 > a.spin_limit) {
                __hip_atomic_fetch_or(ctr_status(a), (uint32_t)STATUS_TIMEOUT, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
                k = 0;
                break;
              }
              __builtin_amdgcn_s_sleep(1);
            }
            it[i] = v;
          }
        }
        break;
      }
    }
  }
  k = __shfl(k, win);
#pragma unroll
  for (int i = 0; i < kClaim; ++i) {
    const uint32_t lo = __shfl((uint32_t)it[i], win), hi = __shfl((uint32_t)(it[i] >> 32), win);
    items[i] = ((u64)hi << 32) | lo;
  }
  return k;
}

// ---------------------------------------------------------------------------------------
// Commutative writes (Sec. 4.1, Sec. 4.7).  The members of a group may run in any order
// but one at a time.  The group's whole state is one 64-bit word: bit 63 = a member holds
// the lock, bit s (s < 63) = member s is ready and waiting for it.  Every change is one
// atomic operation on that word, so a waiter and a releaser cannot miss each other: a
// waiter that finds the lock held stays in the word, and the holder's release hands the
// lock to the lowest waiting member (or clears it when none waits).  A task with several
// commutative data takes their locks one by one in increasing group order, holding the
// earlier ones while it waits for a later one (ordered acquisition: no cycle of waits);
// it is pushed into a ready queue when it holds all of them, and releases them when its
// last part is done.  One thread runs these steps; a grant made for another task is
// followed by the thread that made it.
// ---------------------------------------------------------------------------------------
constexpr u64 kLockBit = 1ull << 63;

// Takes the free lock for the lowest waiting member: its slot + 1, or 0 (lock held, or no
// waiter).
__device__ __forceinline__ uint32_t grant_free_lock(u64* st) {
  u64 cur = __hip_atomic_load(st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    const u64 w = cur & ~kLockBit;
    if ((cur & kLockBit) || !w) return 0u;
    const int s = __ffsll((long long)w) - 1;
    if (__hip_atomic_compare_exchange_strong(st, &cur, (cur | kLockBit) & ~(1ull << s), __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return (uint32_t)s + 1u;
  }
}

// The holder gives the lock up: to the lowest waiting member (its slot + 1 is returned)
// or, with none waiting, back to free (0).
__device__ __forceinline__ uint32_t hand_over_lock(u64* st) {
  u64 cur = __hip_atomic_load(st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    const u64 w = cur & ~kLockBit;
    const int s = w ? __ffsll((long long)w) - 1 : -1;
    const u64 nv = w ? (cur & ~(1ull << s)) : (cur & ~kLockBit);
    if (__hip_atomic_compare_exchange_strong(st, &cur, nv, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return (uint32_t)(s + 1);
  }
}

// Task t, holding the locks of its commutative entries before j, waits for the next ones
// in order; pushes it once it holds them all.  Returns a grant this thread made for
// another member, (group << 6 | slot) + 1, to follow next, or 0.
__device__ uint32_t take_locks_from(const SchedArgs& a, uint32_t t, uint32_t j, int home) {
  const uint32_t c1 = a.coff[t + 1];
  for (uint32_t i = a.coff[t] + j; i < c1; ++i) {
    const uint32_t e = a.cent[i], g = e >> 6, s = e & 63u;
    u64* st = a.gstate + g;
    const u64 old = __hip_atomic_fetch_or(st, 1ull << s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old & kLockBit) return 0u;  // waits in the word: the holder hands it over
    const uint32_t w = grant_free_lock(st);
    if (w == 0u) return 0u;                     // another thread took it (perhaps for t)
    if (w - 1u != s) return ((g << 6) | (w - 1u)) + 1u;  // granted to another member
  }
  push_task(a, t, home);
  return 0u;
}

__device__ void follow_grants(const SchedArgs& a, uint32_t grant, int home) {
  while (grant) {
    const uint32_t e = grant - 1u, m = a.goff[e >> 6] + (e & 63u);
    grant = take_locks_from(a, a.gtask[m], a.gidx[m] + 1u, home);
  }
}

// A task whose last predecessor just finished (descriptor d): pushed, or first through its
// locks.
__device__ __forceinline__ void start_task(const SchedArgs& a, uint32_t t, const TaskDesc& d, int home) {
  if (!a.coff || a.coff[t] == a.coff[t + 1]) {
    push_task(a, t, d, home);
    return;
  }
  follow_grants(a, take_locks_from(a, t, 0u, home), home);
}
__device__ __forceinline__ void start_task(const SchedArgs& a, uint32_t t, int home) {
  start_task(a, t, a.tasks[t], home);
}

// A task whose last part was just released: its locks go to the next waiting members.
__device__ __forceinline__ void drop_locks(const SchedArgs& a, uint32_t t, int home) {
  if (!a.coff) return;
  for (uint32_t i = a.coff[t]; i < a.coff[t + 1]; ++i) {
    const uint32_t g = a.cent[i] >> 6;
    const uint32_t w = hand_over_lock(a.gstate + g);
    if (w) follow_grants(a, ((g << 6) | (w - 1u)) + 1u, home);
  }
}

// The release rounds of XCD x (see the memory-ordering notes above), run by the 64 lanes
// of one wave: each lane takes one ring entry at a time (its parts_left decrement and, for
// a task's last part, the task's locks and done flag); then the successors of every task
// finished in that pass are dealt over the lanes, one (task, successor) pair per lane, so
// a panel's fan-out is decremented and pushed in one round of atomics rather than one
// successor after another.  The j-th successor of a task is pushed into shard (home + j) %
// S: the siblings of a fan-out wait on several queue heads, whose claims proceed in
// parallel, while a lone successor stays in the releasing XCD's own shard (dealt to the
// other shards as well, by its place among the pass's pairs, it left its XCD, and every
// chain task of the overhead study took four times as long).
__device__ __noinline__ void release_rounds(const SchedArgs& a, int x, int home) {
  const int lane = threadIdx.x & 63;
  uint32_t* lock = a.counters + ctr_ring_lock_idx(x);
  uint32_t* tailp = a.counters + ctr_ring_tail_idx(x);
  uint32_t* headp = a.counters + ctr_ring_head_idx(x);
  const uint32_t* ring = a.ring + (size_t)x * a.ring_cap;
  for (;;) {
    uint32_t got = 0u;
    if (lane == 0) {
      uint32_t zero = 0u;
      got = __hip_atomic_compare_exchange_strong(lock, &zero, 1u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)
                ? 1u
                : 0u;
    }
    if (__shfl(got, 0) == 0u) return;  // the holder's next look takes our entries
    uint32_t h = __builtin_amdgcn_readfirstlane(ld_rlx(headp));
    for (;;) {
      const uint32_t t = __builtin_amdgcn_readfirstlane(ld_rlx(tailp));
      if (t == h) break;
      fence_rel();
      const u64 t0 = now_ticks();
      for (uint32_t e0 = h; e0 < t; e0 += 64) {
        const uint32_t e = e0 + (uint32_t)lane;
        uint32_t task = EMPTY32;
        if (e < t) {
          // the slot was reserved by an appender that writes it next: bounded wait
          while ((task = __hip_atomic_load(ring + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == EMPTY32) {
            if (now_ticks() - t0 > a.spin_limit) {
              __hip_atomic_fetch_or(ctr_status(a), (uint32_t)STATUS_TIMEOUT, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
        }
        uint32_t cnt = 0u, first = 0u, last = 0u;
        if (task != EMPTY32) {  // loaded alongside the decrement
          first = a.succ_off[task];
          last = a.succ_off[task + 1];
        }
        if (task != EMPTY32 && sub_rlx(a.parts_left + task, 1u) == 1u) {
          drop_locks(a, task, home);
          if (a.tasks[task].type == SPX_T_STORE) {
            // the release above wrote the STORE's X back: tell the host this matrix is done
            unsigned int* flag = a.mats[a.tasks[task].mat].done_flag;
            if (flag) __hip_atomic_store(flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          }
          cnt = last - first;
        }
        // number the pairs: lane L's finished task owns pairs [off(L), off(L) + cnt(L))
        uint32_t off = cnt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const uint32_t y = __shfl_up(off, d);
          if (lane >= d) off += y;
        }
        const uint32_t total = __shfl(off, 63);
        off -= cnt;
        for (uint32_t i0 = 0; i0 < total; i0 += 64) {
          const uint32_t i = i0 + (uint32_t)lane;
          // the owner of pair i: the last lane whose first pair is at most i (offsets do not
          // decrease over the lanes, and a lane with no pairs shares the next lane's offset)
          int L = 0;
#pragma unroll
          for (int step = 32; step >= 1; step >>= 1)
            if (__shfl(off, L + step) <= i) L += step;
          const uint32_t j = i - __shfl(off, L), q = __shfl(first, L) + j;  // successor j of lane L's task
          if (i < total) {
            const uint32_t s = a.succ[q];
            const TaskDesc ds = a.tasks[s];  // loaded alongside the decrement
            if (sub_rlx(a.pending + s, 1u) == 1u) start_task(a, s, ds, (int)((home + j) % (uint32_t)a.nshards));
          }
        }
      }
      h = t;
      // read-modify-writes, each complete before the next step: the next holder reads
      // this head only after taking the lock this exchange releases
      if (lane == 0) __hip_atomic_exchange(headp, h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // unlock, then look once more: an appender that found the lock taken did so before
    // this unlock, and its tail increment before that
    uint32_t again = 0u;
    if (lane == 0) {
      __hip_atomic_exchange(lock, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      again = ld_rlx(tailp) != h ? 1u : 0u;
    }
    if (__shfl(again, 0) == 0u) return;
  }
}

template <int FAM>
__global__ __launch_bounds__(NT) void sched_kernel(SchedArgs a) {
  __shared__ double lds[LDS_DOUBLES];
  __shared__ u64 s_items[kClaim];
  __shared__ int s_n;
  const int tid = threadIdx.x;
  const int home = blockIdx.x % a.nshards;
  u64 idle = 0, busy = 0;
  // root tasks with commutative accesses take their locks first, spread over the
  // workgroups (the queues hold the other roots already)
  if (tid == 0)
    for (uint32_t r = blockIdx.x; r < a.ncroots; r += gridDim.x) start_task(a, a.croots[r], home);
  for (;;) {
    if (tid < 64) {
      const u64 t0 = now_ticks();
      u64 last_change = t0;
      uint32_t last_taken = 0xffffffffu;
      u64 items[kClaim];
      int n = 0, naps = 0;
      for (;;) {
        bool saw;
        uint32_t taken;
        n = pop_wave(a, home, &saw, &taken, items);
        if (n > 0) break;
        if (saw) {  // the queue emptied under us (or a bounded wait gave up): scan again
          if (__builtin_amdgcn_readfirstlane(ld_rlx(ctr_status(a))) != 0) {
            n = -1;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        const uint32_t status = __builtin_amdgcn_readfirstlane(ld_rlx(ctr_status(a)));
        if (taken >= a.total_parts || status != 0) {
          n = -1;
          break;
        }
        const u64 t = now_ticks();
        if (taken != last_taken) {
          last_taken = taken;
          last_change = t;
        } else if (t - last_change > a.spin_limit) {
          // no part started for the whole spin limit: give up so the kernel ends
          if (tid == 0)
            __hip_atomic_fetch_or(ctr_status(a), (uint32_t)STATUS_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          n = -1;
          break;
        }
        // back off (up to about 1.7 us) while the queues stay empty: every scan is 64
        // uncached loads, and hundreds of idle workgroups polling would take memory
        // bandwidth from the ones running the critical path
        if (naps < 5) ++naps;
        for (int z = 0; z < (1 << naps); ++z) __builtin_amdgcn_s_sleep(2);
      }
      if (tid == 0) {
        // a popped task was pushed when its last predecessor's decrement took the counter
        // to zero, so the wait below ends at once; it is bounded all the same
        const u64 tw = now_ticks();
        for (int i = 0; i < n; ++i) {
          const uint32_t* pend = a.pending + (uint32_t)(items[i] >> 16);
          while (ld_rlx(pend) != 0u) {
            if (now_ticks() - tw > a.spin_limit) {
              __hip_atomic_fetch_or(ctr_status(a), (uint32_t)STATUS_TIMEOUT, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
              n = -1;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
          if (n < 0) break;
          s_items[i] = items[i];
        }
        if (n > 0) fence_acq();
        s_n = n;
        idle += now_ticks() - t0;
      }
    }
    __syncthreads();
    const int n = s_n;
    if (n < 0) break;
    for (int i = 0; i < n; ++i) {
      const u64 item = s_items[i];
      const uint32_t task = (uint32_t)(item >> 16), part = (uint32_t)(item & 0xffff);
      const u64 tb = now_ticks();
      run_part<FAM>(a, task, part, lds);
      __syncthreads();
      if (tid == 0) {
        const u64 te = now_ticks();
        busy += te - tb;
        if (a.trace) {
          const uint32_t k = atomicAdd(a.trace_idx, 1u);
          if (k < a.total_parts) {
            a.trace[4 * k + 0] = task;
            a.trace[4 * k + 1] = part | ((u64)blockIdx.x << 16) | ((u64)a.tasks[task].type << 32);
            a.trace[4 * k + 2] = tb;
            a.trace[4 * k + 3] = te;
          }
        }
      }
    }
    // hand the claim's parts to this XCD's release rounds (wave 0; the barrier above
    // waited for every wave's stores)
    if (tid < 64) {
      const int x = xcd_id();
      uint32_t* ring = a.ring + (size_t)x * a.ring_cap;
      uint32_t slot = 0u;
      if (tid == 0)
        slot = __hip_atomic_fetch_add(a.counters + ctr_ring_tail_idx(x), (uint32_t)n, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
      slot = __shfl(slot, 0);
      if (tid < n)
        __hip_atomic_store(ring + slot + tid, (uint32_t)(s_items[tid] >> 16), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      release_rounds(a, x, home);
    }
  }
  if (tid == 0 && a.wg_cycles) {
    a.wg_cycles[2 * blockIdx.x + 0] = busy;
    a.wg_cycles[2 * blockIdx.x + 1] = idle;
  }
}

// One task, part blockIdx.x per workgroup (tests of the tile kernels).
__global__ __launch_bounds__(NT) void one_task_kernel(SchedArgs a) {
  __shared__ double lds[LDS_DOUBLES];
  run_part_chol(a, 0, blockIdx.x, lds);
}

__global__ __launch_bounds__(NT) void tile_inverses_kernel(const double* l, int b, double* dinv) {
  __shared__ double lds[4 * 2048];
  tile_inverses(l, b, dinv, lds);
}

// Per-launch state from the cached static image: counters of unfinished predecessors
// and parts, cleared queues and counters (the root parts are written by roots_kernel,
// launched after this one).
__global__ void sched_init_kernel(uint32_t* pending, const uint32_t* indeg, uint32_t* parts_left,
                                  const uint32_t* nparts, uint32_t ntasks, u64* queue, uint32_t queue_len,
                                  uint32_t* counters, const uint32_t* counters0, uint32_t ncounters,
                                  uint32_t* ring, uint32_t ring_len, u64* gstate, uint32_t ngroups, int32_t* info,
                                  int ninfo, uint32_t* trace_idx) {
  const uint32_t stride = gridDim.x * blockDim.x;
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  for (uint32_t t = g; t < ntasks; t += stride) {
    pending[t] = indeg[t];
    parts_left[t] = nparts[t];
  }
  for (uint32_t t = g; t < queue_len; t += stride) queue[t] = EMPTY;
  for (uint32_t t = g; t < ncounters; t += stride) counters[t] = counters0[t];
  for (uint32_t t = g; t < ring_len; t += stride) ring[t] = EMPTY32;
  for (uint32_t t = g; t < ngroups; t += stride) gstate[t] = 0ull;
  for (uint32_t t = g; t < (uint32_t)ninfo; t += stride) info[t] = INT_MAX;
  if (g == 0 && trace_idx) *trace_idx = 0;
}

__global__ void roots_kernel(u64* queue, const u64* roots, uint32_t nroots) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < nroots; r += stride) queue[roots[2 * r]] = roots[2 * r + 1];
}

// ---------------------------------------------------------------------------------------
// Packing between the caller's dense row-major matrix and the tile storage.
// One workgroup per 64x64 (or b x b if b < 64) sub-block of a lower tile, transposed
// through LDS so both the row-major reads and the column-major writes are coalesced.
// Rows/columns >= n form an identity border (padding).
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void pack_kernel(const double* __restrict__ A, int64_t lda, int64_t n, DevMat m) {
  __shared__ double s[64 * 65];
  const int nt = m.nt, b = m.b;
  const int S = b < 64 ? b : 64, per = b / S;
  const int ti = blockIdx.x / nt, tj = blockIdx.x % nt;
  if (tj > ti) return;
  pack_block(A, lda, n, m, ti, tj, blockIdx.y / per, blockIdx.y % per, S, s);
}

// All tiles of a dense row-major n x n matrix (or of its transpose): one workgroup per
// 64x64 (or b x b) sub-block of a tile, through LDS so the row-major reads and the
// column-major tile writes are both coalesced.  Entries beyond n are zero.
__global__ __launch_bounds__(NT) void pack_full_kernel(const double* __restrict__ src, int64_t ld, int64_t n,
                                                       double* __restrict__ tiles, int b, int nt, int trans) {
  __shared__ double s[64 * 65];
  const int S = b < 64 ? b : 64, per = b / S;
  const int ti = blockIdx.x / nt, tj = blockIdx.x % nt;
  const int si = blockIdx.y / per, sj = blockIdx.y % per;
  const int64_t R0 = (int64_t)ti * b + si * S, C0 = (int64_t)tj * b + sj * S;  // of the packed matrix
  // s[x * 65 + y]: element (R0 + (trans ? y : x), C0 + (trans ? x : y)) where (x, y) walks the
  // source row by row
  for (int e = threadIdx.x; e < S * S; e += NT) {
    const int x = e / S, y = e % S;
    const int64_t sr = trans ? C0 + x : R0 + x, sc = trans ? R0 + y : C0 + y;  // source row, column
    s[x * 65 + y] = (sr < n && sc < n) ? src[sr * ld + sc] : 0.0;
  }
  __syncthreads();
  double* T = tiles + ((size_t)ti * nt + tj) * (size_t)b * b;
  for (int e = threadIdx.x; e < S * S; e += NT) {
    const int c = e / S, r = e % S;  // tile column, row (r fastest: coalesced writes)
    T[(size_t)(sj * S + c) * b + si * S + r] = trans ? s[c * 65 + r] : s[r * 65 + c];
  }
}

__global__ __launch_bounds__(NT) void unpack_full_kernel(const double* __restrict__ tiles, int b, int nt, int64_t n,
                                                         double* __restrict__ dst, int64_t ld) {
  __shared__ double s[64 * 65];
  const int S = b < 64 ? b : 64, per = b / S;
  const int ti = blockIdx.x / nt, tj = blockIdx.x % nt;
  const int si = blockIdx.y / per, sj = blockIdx.y % per;
  const int64_t R0 = (int64_t)ti * b + si * S, C0 = (int64_t)tj * b + sj * S;
  if (R0 >= n || C0 >= n) return;
  const double* T = tiles + ((size_t)ti * nt + tj) * (size_t)b * b;
  for (int e = threadIdx.x; e < S * S; e += NT) {
    const int c = e / S, r = e % S;
    s[r * 65 + c] = T[(size_t)(sj * S + c) * b + si * S + r];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < S * S; e += NT) {
    const int r = e / S, c = e % S;
    if (R0 + r < n && C0 + c < n) dst[(R0 + r) * ld + C0 + c] = s[r * 65 + c];
  }
}

// Diagonally dominant SPD test matrix (row-major n x n, both triangles): off-diagonal
// entries uniform in [-1, 1) / n from a hash of (min(i,j), max(i,j), seed), diagonal 2.
__global__ void spd_fill_kernel(double* __restrict__ A, int64_t n, uint32_t seed) {
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e % n;
    if (i == j) {
      A[e] = 2.0;
      continue;
    }
    uint64_t h = ((uint64_t)(i < j ? i : j) << 32) ^ (uint64_t)(i < j ? j : i) ^ ((uint64_t)seed << 56);
    h ^= h >> 33;
    h *= 0xff51afd7ed558ccdull;
    h ^= h >> 33;
    h *= 0xc4ceb9fe1a85ec53ull;
    h ^= h >> 33;
    A[e] = ((double)(h >> 11) * 0x1.0p-53 * 2.0 - 1.0) / (double)n;
  }
}

__global__ __launch_bounds__(NT) void unpack_kernel(DevMat m, int64_t n, double* __restrict__ L, int64_t ldl) {
  __shared__ double s[64][65];
  const int nt = m.nt, b = m.b;
  const int S = b < 64 ? b : 64, per = b / S;
  const int ti = blockIdx.x / nt, tj = blockIdx.x % nt;
  const int si = blockIdx.y / per, sj = blockIdx.y % per;
  const int64_t R0 = (int64_t)ti * b + si * S, C0 = (int64_t)tj * b + sj * S;
  if (R0 >= n || C0 >= n) return;
  if (tj <= ti) {
    const double* T = tile_ptr(m, ti, tj);
    for (int e = threadIdx.x; e < S * S; e += NT) {
      const int cc = e / S, rr = e % S;
      s[rr][cc] = T[(size_t)(sj * S + cc) * b + si * S + rr];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < S * S; e += NT) {
    const int rr = e / S, cc = e % S;
    const int64_t R = R0 + rr, C = C0 + cc;
    if (R < n && C < n) L[R * ldl + C] = (tj <= ti && R >= C) ? s[rr][cc] : 0.0;
  }
}

// Right-hand sides: row-major n x nrhs <-> column-major n_pad x nrhs (zero padding),
// optionally scaling row r by scale[r].
__global__ void rhs_in_kernel(const double* __restrict__ B, int64_t ldb, int64_t n, int64_t nrhs,
                              double* __restrict__ y, int64_t n_pad, const double* __restrict__ scale) {
  const int64_t total = n_pad * nrhs;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = e / n_pad, r = e % n_pad;
    const double v = r < n ? B[r * ldb + q] : 0.0;
    y[e] = (scale && r < n) ? v * scale[r] : v;
  }
}
__global__ void rhs_out_kernel(const double* __restrict__ y, int64_t n_pad, int64_t n, int64_t nrhs,
                               double* __restrict__ X, int64_t ldx, int accumulate, const double* __restrict__ scale) {
  const int64_t total = n * nrhs;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / nrhs, q = e % nrhs;
    const double v = scale ? y[q * n_pad + r] * scale[r] : y[q * n_pad + r];
    if (accumulate)
      X[r * ldx + q] += v;
    else
      X[r * ldx + q] = v;
  }
}

__global__ void diag_scale_kernel(const double* __restrict__ A, int64_t lda, int64_t n, double* __restrict__ d,
                                  int64_t n_pad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pad; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = i < n ? 1.0 / sqrt(A[i * lda + i]) : 1.0;
}

// Thread g (of nthr, a multiple of q) sums U .* V over the elements g, g + nthr, ...: all
// of one column (g mod q).
__global__ void dot_cols_kernel(int64_t total, int64_t nthr, const double* __restrict__ U,
                                const double* __restrict__ V, double* __restrict__ partial) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nthr) return;
  double acc = 0.0;
  for (int64_t e = g; e < total; e += nthr) acc += U[e] * V[e];
  partial[g] = acc;
}

__global__ void axpy_cols_kernel(int64_t total, int64_t q, const double* __restrict__ alpha,
                                 const double* __restrict__ X, double* __restrict__ Y, int mode) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const double a = alpha[e % q];
    Y[e] = mode == 0 ? Y[e] + a * X[e] : X[e] + a * Y[e];
  }
}

// ---------------------------------------------------------------------------------------
// Residual r = b - A x for the dense symmetric A (lower triangle of a row-major array),
// 64 rows per workgroup; and per-column maxima of |r|, |x|, |b| for the backward error.
// Row i's entries left of the block are read along the row; the rest along the column
// (A(j, i), j >= i), so every load is a contiguous strip.
// stats: per column q: [3q] max|r|, [3q+1] max|x|, [3q+2] max|b| (as non-negative
// doubles compared through their bit patterns); the last slot holds ||A||_inf.
// ---------------------------------------------------------------------------------------
// Right-hand sides per pass of the residual kernels over A (each pass reads the matrix).
constexpr int kResQ = 16;

__device__ __forceinline__ void atomic_max_nonneg(double* p, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ void residual_rows(int64_t n, const double* __restrict__ A, int64_t lda, int64_t nrhs,
                              const double* __restrict__ X, int64_t ldx, const double* __restrict__ Bv, int64_t ldb,
                              double* __restrict__ R, double* __restrict__ stats, int64_t i0,
                              double (*part)[64][kResQ + 1]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int Q = kResQ;  // right-hand sides per pass over A
  for (int64_t q0 = 0; q0 < nrhs; q0 += Q) {
    const int nq = (nrhs - q0) < Q ? (int)(nrhs - q0) : Q;
    double acc[Q + 1];  // Q right-hand sides + the absolute row sum
#pragma unroll
    for (int q = 0; q <= Q; ++q) acc[q] = 0.0;
    const int64_t i = i0 + lane;
    // part 1: columns j < i0, read along rows.  Wave w takes rows i0 + w + 4 t (t < 16),
    // four at a time; the rows of X for 256 columns at a time are staged in LDS (in the
    // buffer of the closing reduction, which has the same size) and shared by the waves,
    // so X is read once per four rows instead of once per row and never gathered from
    // global memory.  Lane l sums the columns j = l mod 64 in increasing order, and the
    // lanes are reduced with the same butterfly, as a row-by-row loop would.
    {
      constexpr int CH = 256, XS = Q + 1, RG = 2;
      static_assert(CH * XS <= 4 * 64 * (Q + 1), "a chunk of X fits the reduction buffer");
      LDSAS double* xs = lp(&part[0][0][0]);
      for (int g = 0; g < 16 / RG; ++g) {
        double sp[RG][Q + 1];
#pragma unroll
        for (int t = 0; t < RG; ++t)
#pragma unroll
          for (int q = 0; q <= Q; ++q) sp[t][q] = 0.0;
        for (int64_t j0 = 0; j0 < i0; j0 += CH) {
          __syncthreads();  // the previous chunk (or the buffer's earlier use) is done with
          {
            const int t = threadIdx.x;
            const int64_t j = j0 + t;
            if (j < i0) {
#pragma unroll
              for (int q = 0; q < Q; ++q) xs[t * XS + q] = q < nq ? X[j * ldx + q0 + q] : 0.0;
            }
          }
          __syncthreads();
          double a[CH / 64][RG];  // every load of the chunk issued before the first use
#pragma unroll
          for (int k = 0; k < CH / 64; ++k)
#pragma unroll
            for (int t = 0; t < RG; ++t) {
              const int64_t ii = i0 + wave + 4 * (RG * g + t), j = j0 + lane + 64 * k;
              a[k][t] = (ii < n && j < i0) ? A[ii * lda + j] : 0.0;
            }
#pragma unroll
          for (int k = 0; k < CH / 64; ++k) {
            const int c = lane + 64 * k;
            if (j0 + c < i0) {
              double xv[Q];
#pragma unroll
              for (int q = 0; q < Q; ++q) xv[q] = xs[c * XS + q];
#pragma unroll
              for (int t = 0; t < RG; ++t) {
                const int64_t ii = i0 + wave + 4 * (RG * g + t);
                if (ii < n) {
                  const double aij = a[k][t];
#pragma unroll
                  for (int q = 0; q < Q; ++q)
                    if (q < nq) sp[t][q] += aij * xv[q];
                  sp[t][Q] += fabs(aij);
                }
              }
            }
          }
        }
#pragma unroll
        for (int t = 0; t < RG; ++t) {
          const int rr = wave + 4 * (RG * g + t);
          if (i0 + rr >= n) continue;
#pragma unroll
          for (int q = 0; q <= Q; ++q)
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) sp[t][q] += __shfl_xor(sp[t][q], off);
          if (lane == rr) {
#pragma unroll
            for (int q = 0; q <= Q; ++q) acc[q] += sp[t][q];
          }
        }
      }
      __syncthreads();  // the reduction buffer is free again
    }
    // part 2: columns j >= i0; lane owns row i, wave w takes j = i0 + w, i0 + w + 4, ...
    // in increasing order.  X again comes through LDS 256 rows at a time (read by a wave
    // at one address per row: a broadcast), and the loads of A (row j's 64 entries of the
    // block, contiguous) are issued eight rows at a time, so a wave has eight in flight
    // instead of waiting for each.
    {
      constexpr int CH = 256, XS = Q + 1, U = 8;
      LDSAS double* xs = lp(&part[0][0][0]);
      for (int64_t j0 = i0; j0 < n; j0 += CH) {
        __syncthreads();
        {
          const int t = threadIdx.x;
          const int64_t j = j0 + t;
          if (j < n) {
#pragma unroll
            for (int q = 0; q < Q; ++q) xs[t * XS + q] = q < nq ? X[j * ldx + q0 + q] : 0.0;
          }
        }
        __syncthreads();
        if (i < n) {
          for (int k0 = wave; k0 < CH; k0 += 4 * U) {
            double a[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const int64_t j = j0 + k0 + 4 * u;
              a[u] = (k0 + 4 * u < CH && j < n) ? ((j >= i) ? A[j * lda + i] : A[i * lda + j]) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const int c = k0 + 4 * u;
              if (c < CH && j0 + c < n) {
                const double aij = a[u];
#pragma unroll
                for (int q = 0; q < Q; ++q)
                  if (q < nq) acc[q] += aij * xs[c * XS + q];
                acc[Q] += fabs(aij);
              }
            }
          }
        }
      }
      __syncthreads();  // the buffer is free for the partial sums
    }
#pragma unroll
    for (int q = 0; q <= Q; ++q) part[wave][lane][q] = acc[q];
    __syncthreads();
    if (wave == 0) {
      // the block's 64 rows: residuals, then the maxima of |r|, |x|, |b| per right-hand
      // side and of the absolute row sums reduced across the wave on their bit patterns (as
      // atomic_max_nonneg compares them; a NaN stays the maximum), so each workgroup makes
      // one atomic per statistic (a max: the order does not change the result).  One
      // column at a time, its sums read back from LDS, to keep few registers live.
      auto wave_max = [&](double v) {
        unsigned long long bits = (unsigned long long)__double_as_longlong(v);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
          const unsigned long long o = __shfl_xor(bits, off);
          bits = o > bits ? o : bits;
        }
        return __longlong_as_double((long long)bits);
      };
      for (int q = 0; q <= nq; ++q) {
        const int c = q < nq ? q : Q;  // the last round: the absolute row sums
        double v0 = 0.0, v1 = 0.0, v2 = 0.0;
        if (i < n) {
          const double tot = part[0][lane][c] + part[1][lane][c] + part[2][lane][c] + part[3][lane][c];
          if (q < nq) {
            const double r = Bv[i * ldb + q0 + q] - tot;
            R[i * nrhs + q0 + q] = r;
            v0 = fabs(r);
            v1 = fabs(X[i * ldx + q0 + q]);
            v2 = fabs(Bv[i * ldb + q0 + q]);
          } else {
            v0 = tot;
          }
        }
        v0 = wave_max(v0);
        if (q < nq) {
          v1 = wave_max(v1);
          v2 = wave_max(v2);
          if (lane == 0) {
            atomic_max_nonneg(stats + 3 * (q0 + q) + 0, v0);
            atomic_max_nonneg(stats + 3 * (q0 + q) + 1, v1);
            atomic_max_nonneg(stats + 3 * (q0 + q) + 2, v2);
          }
        } else if (lane == 0 && q0 == 0) {
          atomic_max_nonneg(stats + 3 * nrhs, v0);
        }
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(NT) void residual_kernel(int64_t n, const double* __restrict__ A, int64_t lda,
                                                      int64_t nrhs, const double* __restrict__ X, int64_t ldx,
                                                      const double* __restrict__ Bv, int64_t ldb,
                                                      double* __restrict__ R, double* __restrict__ stats) {
  __shared__ double part[4][64][kResQ + 1];
  residual_rows(n, A, lda, nrhs, X, ldx, Bv, ldb, R, stats, (int64_t)blockIdx.x * 64, part);
}

__global__ __launch_bounds__(NT) void residual_batched_kernel(const ResDesc* __restrict__ d,
                                                              const uint32_t* __restrict__ prefix, int count) {
  __shared__ double part[4][64][kResQ + 1];
  const uint32_t blk = blockIdx.x;
  int lo = 0, hi = count - 1;  // last m with prefix[m] <= blk
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= blk) lo = mid; else hi = mid - 1;
  }
  const ResDesc r = d[lo];
  residual_rows(r.n, r.A, r.lda, r.nrhs, r.X, r.ldx, r.B, r.ldb, r.R, r.stats, (int64_t)(blk - prefix[lo]) * 64,
                part);
}

// ---------------------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------------------
static int hip_ok(hipError_t e, const char* what) {
  if (e == hipSuccess) return SPX_OK;
  // a launch that cannot get its scratch memory reports out of memory: the caller may retry smaller
  return failf(e == hipErrorOutOfMemory ? SPX_ENOMEM : SPX_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------------------------------
// Scratch memory of the allocation-free entry point (spx_potrs_noalloc): one array per
// device, part of the loaded code object, held until the process ends.  Host code never
// uses the array's name as an address (on the host it is only a stand-in for the symbol):
// the device address of each GPU's copy is looked up once, with that device current, and
// kept here.
// ---------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(SPX_EINVAL, "scratch: device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return SPX_OK;
  int cur = -1;
  if (int rc = hip_ok(hipGetDevice(&cur), "hipGetDevice")) return rc;
  if (cur != device) return fail(SPX_EINVAL, "scratch: the device must be current");
  void* p = nullptr;
  if (int rc = hip_ok(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)")) return rc;
  if (!p) return fail(SPX_EDEVICE, "hipGetSymbolAddress(scratch) returned null");
  g_scratch_ptr[device] = p;
  return SPX_OK;
}

int scratch_get(int device, void** ptr) {
  if (device < 0 || device >= kMaxDevices) return fail(SPX_EINVAL, "scratch: device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) return fail(SPX_EINVAL, "scratch: not set up on this device");
  *ptr = g_scratch_ptr[device];
  return SPX_OK;
}

int launch_pack(const double* dA, int64_t lda, int64_t n, const DevMat& m, void* stream) {
  const int S = m.b < 64 ? m.b : 64, per = m.b / S;
  dim3 grid((unsigned)(m.nt * m.nt), (unsigned)(per * per));
  hipLaunchKernelGGL(pack_kernel, grid, dim3(NT), 0, (hipStream_t)stream, dA, lda, n, m);
  return hip_ok(hipGetLastError(), "pack_kernel");
}

int launch_pack_full(const double* src, int64_t ld, int64_t n, double* tiles, int b, int nt, int trans, void* stream) {
  const int S = b < 64 ? b : 64, per = b / S;
  dim3 grid((unsigned)(nt * nt), (unsigned)(per * per));
  hipLaunchKernelGGL(pack_full_kernel, grid, dim3(NT), 0, (hipStream_t)stream, src, ld, n, tiles, b, nt, trans);
  return hip_ok(hipGetLastError(), "pack_full_kernel");
}

int launch_unpack_full(const double* tiles, int b, int nt, int64_t n, double* dst, int64_t ld, void* stream) {
  const int S = b < 64 ? b : 64, per = b / S;
  dim3 grid((unsigned)(nt * nt), (unsigned)(per * per));
  hipLaunchKernelGGL(unpack_full_kernel, grid, dim3(NT), 0, (hipStream_t)stream, tiles, b, nt, n, dst, ld);
  return hip_ok(hipGetLastError(), "unpack_full_kernel");
}

int launch_spd_fill(double* A, int64_t n, uint32_t seed, void* stream) {
  hipLaunchKernelGGL(spd_fill_kernel, dim3(1024), dim3(NT), 0, (hipStream_t)stream, A, n, seed);
  return hip_ok(hipGetLastError(), "spd_fill_kernel");
}

int launch_unpack(const DevMat& m, int64_t n, double* dL, int64_t ldl, void* stream) {
  const int S = m.b < 64 ? m.b : 64, per = m.b / S;
  dim3 grid((unsigned)(m.nt * m.nt), (unsigned)(per * per));
  hipLaunchKernelGGL(unpack_kernel, grid, dim3(NT), 0, (hipStream_t)stream, m, n, dL, ldl);
  return hip_ok(hipGetLastError(), "unpack_kernel");
}

int launch_rhs_in(const double* dB, int64_t ldb, int64_t n, int64_t nrhs, double* rhs, int64_t n_pad,
                  const double* scale, void* stream) {
  hipLaunchKernelGGL(rhs_in_kernel, dim3(1024), dim3(NT), 0, (hipStream_t)stream, dB, ldb, n, nrhs, rhs, n_pad, scale);
  return hip_ok(hipGetLastError(), "rhs_in_kernel");
}

int launch_diag_scale(const double* dA, int64_t lda, int64_t n, double* d, int64_t n_pad, void* stream) {
  hipLaunchKernelGGL(diag_scale_kernel, dim3(256), dim3(NT), 0, (hipStream_t)stream, dA, lda, n, d, n_pad);
  return hip_ok(hipGetLastError(), "diag_scale_kernel");
}

int launch_dot_cols(int64_t n, int64_t q, const double* U, const double* V, double* partial, int* nthreads,
                    void* stream) {
  const int64_t cap = 256 * NT;
  if (q < 1 || q > cap) return fail(SPX_EINVAL, "dot_cols: too many columns");
  const int64_t nthr = (cap / q) * q;
  *nthreads = (int)nthr;
  hipLaunchKernelGGL(dot_cols_kernel, dim3((unsigned)((nthr + NT - 1) / NT)), dim3(NT), 0, (hipStream_t)stream,
                     n * q, nthr, U, V, partial);
  return hip_ok(hipGetLastError(), "dot_cols_kernel");
}

int launch_axpy_cols(int64_t n, int64_t q, const double* alpha, const double* X, double* Y, int mode, void* stream) {
  hipLaunchKernelGGL(axpy_cols_kernel, dim3(1024), dim3(NT), 0, (hipStream_t)stream, n * q, q, alpha, X, Y, mode);
  return hip_ok(hipGetLastError(), "axpy_cols_kernel");
}

int launch_rhs_out(const double* rhs, int64_t n_pad, int64_t n, int64_t nrhs, double* dX, int64_t ldx, int accumulate,
                   const double* scale, void* stream) {
  hipLaunchKernelGGL(rhs_out_kernel, dim3(1024), dim3(NT), 0, (hipStream_t)stream, rhs, n_pad, n, nrhs, dX, ldx,
                     accumulate, scale);
  return hip_ok(hipGetLastError(), "rhs_out_kernel");
}

int sched_max_wg(int device, int* per_cu, int* num_cu) {
  int blocks = 0;
  if (int rc = hip_ok(hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, sched_kernel<FAM_CHOL>, NT, 0),
                      "hipOccupancyMaxActiveBlocksPerMultiprocessor"))
    return rc;
  int cus = 0;
  if (int rc = hip_ok(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device),
                      "hipDeviceGetAttribute"))
    return rc;
  *per_cu = blocks;
  *num_cu = cus;
  return SPX_OK;
}

int launch_tile_inverses(const double* l, int b, double* dinv, void* stream) {
  hipLaunchKernelGGL(tile_inverses_kernel, dim3(1), dim3(NT), 0, (hipStream_t)stream, l, b, dinv);
  return hip_ok(hipGetLastError(), "tile_inverses_kernel");
}

int launch_one_task(const SchedArgs& a, int nparts, void* stream) {
  hipLaunchKernelGGL(one_task_kernel, dim3(nparts), dim3(NT), 0, (hipStream_t)stream, a);
  return hip_ok(hipGetLastError(), "one_task_kernel");
}

int launch_sched(const SchedArgs& a, int num_wg, void* stream, int family) {
  if (family == FAM_GEMM)
    hipLaunchKernelGGL(sched_kernel<FAM_GEMM>, dim3(num_wg), dim3(NT), 0, (hipStream_t)stream, a);
  else if (family == FAM_SPIN)
    hipLaunchKernelGGL(sched_kernel<FAM_SPIN>, dim3(num_wg), dim3(NT), 0, (hipStream_t)stream, a);
  else
    hipLaunchKernelGGL(sched_kernel<FAM_CHOL>, dim3(num_wg), dim3(NT), 0, (hipStream_t)stream, a);
  return hip_ok(hipGetLastError(), "sched_kernel");
}

int launch_sched_init_full(uint32_t* pending, const uint32_t* indeg, uint32_t* parts_left, const uint32_t* nparts,
                           uint32_t ntasks, unsigned long long* queue, uint32_t queue_len,
                           const unsigned long long* roots, uint32_t nroots, uint32_t* counters,
                           const uint32_t* counters0, uint32_t ncounters, uint32_t* ring, uint32_t ring_len,
                           unsigned long long* gstate, uint32_t ngroups, int32_t* info, int ninfo,
                           uint32_t* trace_idx, void* stream) {
  hipLaunchKernelGGL(sched_init_kernel, dim3(1024), dim3(NT), 0, (hipStream_t)stream, pending, indeg, parts_left,
                     nparts, ntasks, queue, queue_len, counters, counters0, ncounters, ring, ring_len, gstate,
                     ngroups, info, ninfo, trace_idx);
  const int rc = hip_ok(hipGetLastError(), "sched_init_kernel");
  if (rc) return rc;
  hipLaunchKernelGGL(roots_kernel, dim3(256), dim3(NT), 0, (hipStream_t)stream, queue, roots, nroots);
  return hip_ok(hipGetLastError(), "roots_kernel");
}

int launch_backward_error(int64_t n, const double* dA, int64_t lda, int64_t nrhs, const double* dX, int64_t ldx,
                          const double* dB, int64_t ldb, double* dR, double* dstats, void* stream) {
  const unsigned grid = (unsigned)((n + 63) / 64);
  hipLaunchKernelGGL(residual_kernel, dim3(grid), dim3(NT), 0, (hipStream_t)stream, n, dA, lda, nrhs, dX, ldx, dB,
                     ldb, dR, dstats);
  return hip_ok(hipGetLastError(), "residual_kernel");
}

int launch_backward_error_batched(const ResDesc* d, const uint32_t* prefix, int count, uint32_t nblocks,
                                  void* stream) {
  if (nblocks == 0) return SPX_OK;
  hipLaunchKernelGGL(residual_batched_kernel, dim3(nblocks), dim3(NT), 0, (hipStream_t)stream, d, prefix, count);
  return hip_ok(hipGetLastError(), "residual_batched_kernel");
}

}  // namespace spx
