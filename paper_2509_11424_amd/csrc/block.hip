// Tall-skinny products and CholeskyQR of blocks of level vectors (layout in
// block.h).  A product C = A^H B stages 32 rows of a 32-column tile of both
// operands in LDS per pass and accumulates a 32 x 32 output tile (2 x 2 per
// thread) over a chunk of rows; the chunk partials are summed in a fixed
// order, so results are deterministic.  CholeskyQR forms the Gram matrix on
// the GPU, factors it and inverts the k x k triangle on the host in FP64, and
// multiplies V by the inverse in place: applied twice it gives the unique Q
// with positive real diag(R) (the Q of modified Gram-Schmidt, up to rounding).
#include <cmath>

#include "block.h"

namespace mgm {

namespace {

constexpr int kTile = 32;       // output tile edge of the tall-skinny product
constexpr int kRowsLds = 32;    // rows staged per LDS pass
constexpr int kChunksMax = 256; // row chunks (partial sums) per product

// part[chunk][i][j] = sum over the chunk's rows of conj(A[row][i]) B[row][j]
// (A: rows x ka, B: rows x kb, row-major); grid (tiles_i * tiles_j, chunks).
__global__ __launch_bounds__(256) void k_ts_ahb(const double2* __restrict__ A, int ka, const double2* __restrict__ B,
                                               int kb, int64_t rows, int64_t rows_per_chunk, int tiles_j,
                                               double2* __restrict__ part) {
  __shared__ double2 sA[kRowsLds][kTile];
  __shared__ double2 sB[kRowsLds][kTile];
  const int ti = blockIdx.x / tiles_j, tj = blockIdx.x % tiles_j;
  const int i0 = ti * kTile, j0 = tj * kTile;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t r_begin = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t r_end = r_begin + rows_per_chunk < rows ? r_begin + rows_per_chunk : rows;
  double2 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) acc[a][b] = make_double2(0.0, 0.0);
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kRowsLds) {
    __syncthreads();
    for (int e = threadIdx.x; e < kRowsLds * kTile; e += 256) {
      const int rr = e / kTile, cc = e % kTile;
      const int64_t row = r0 + rr;
      const bool in_row = row < r_end;
      sA[rr][cc] = (in_row && i0 + cc < ka) ? A[row * ka + i0 + cc] : make_double2(0.0, 0.0);
      sB[rr][cc] = (in_row && j0 + cc < kb) ? B[row * kb + j0 + cc] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < kRowsLds; rr++) {
      const double2 a0 = sA[rr][2 * ty], a1 = sA[rr][2 * ty + 1];
      const double2 b0 = sB[rr][2 * tx], b1 = sB[rr][2 * tx + 1];
      // conj(a) * b
      acc[0][0].x += a0.x * b0.x + a0.y * b0.y;
      acc[0][0].y += a0.x * b0.y - a0.y * b0.x;
      acc[0][1].x += a0.x * b1.x + a0.y * b1.y;
      acc[0][1].y += a0.x * b1.y - a0.y * b1.x;
      acc[1][0].x += a1.x * b0.x + a1.y * b0.y;
      acc[1][0].y += a1.x * b0.y - a1.y * b0.x;
      acc[1][1].x += a1.x * b1.x + a1.y * b1.y;
      acc[1][1].y += a1.x * b1.y - a1.y * b1.x;
    }
  }
  double2* out = part + (size_t)blockIdx.y * ka * kb;
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) {
      const int i = i0 + 2 * ty + a, j = j0 + 2 * tx + b;
      if (i < ka && j < kb) out[(size_t)i * kb + j] = acc[a][b];
    }
}

// C[e] = sum_chunk part[chunk][e], chunks in order
__global__ void k_sum_chunks(const double2* __restrict__ part, int64_t m, int chunks, double2* __restrict__ C) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  double2 s = make_double2(0.0, 0.0);
  for (int c = 0; c < chunks; c++) {
    const double2 v = part[(size_t)c * m + e];
    s.x += v.x;
    s.y += v.y;
  }
  C[e] = s;
}

// W[row][:] <- W[row][:] M in place (W: rows x k, M: k x k, row-major); a
// block stages rows_pb rows in LDS (dynamic, rows_pb * k entries).
__global__ __launch_bounds__(256) void k_rowmul(double2* __restrict__ W, int k, int64_t rows, int rows_pb,
                                               const double2* __restrict__ M) {
  extern __shared__ double2 sW[];
  const int64_t r0 = (int64_t)blockIdx.x * rows_pb;
  const int nr = (int)(rows - r0 < rows_pb ? rows - r0 : rows_pb);
  for (int e = threadIdx.x; e < nr * k; e += 256) sW[e] = W[r0 * k + e];
  __syncthreads();
  for (int e = threadIdx.x; e < nr * k; e += 256) {
    const int r = e / k, j = e % k;
    double sx = 0.0, sy = 0.0;
    for (int i = 0; i < k; i++) {
      const double2 w = sW[r * k + i], m = M[(size_t)i * k + j];
      sx += w.x * m.x - w.y * m.y;
      sy += w.x * m.y + w.y * m.x;
    }
    W[r0 * k + e] = make_double2(sx, sy);
  }
}

// out[(d*V + s)*b + j] = sign(d) V[(d*V + s)*k + c0 + j], sign = -1 on the
// lower spin half when g5 (Gamma5 of the fine lattice: dof = 3*spin + colour)
__global__ void k_gather_cols(const double2* __restrict__ Vb, int k, int c0, int b, int64_t nsite, int dof, int g5,
                              double2* __restrict__ out) {
  const int64_t n = nsite * dof * b;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e / b;
    const int j = (int)(e - row * b);
    double2 v = Vb[row * k + c0 + j];
    if (g5 && (int)(row / nsite) >= dof / 2) v = make_double2(-v.x, -v.y);
    out[e] = v;
  }
}

__global__ void k_scatter_cols(const double2* __restrict__ in, int k, int c0, int b, int64_t rows,
                               double2* __restrict__ Vb) {
  const int64_t n = rows * b;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e / b;
    const int j = (int)(e - row * b);
    Vb[row * k + c0 + j] = in[e];
  }
}

unsigned grid_of(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b < 65536 * 4 ? b : 65536 * 4);
}

}  // namespace

void blk_ahb(Context* c, const double2* A, int ka, const double2* B, int kb, int64_t rows, double2* part,
             size_t part_cap, double2* C) {
  const int ti = (ka + kTile - 1) / kTile, tj = (kb + kTile - 1) / kTile;
  int64_t chunks = std::max<int64_t>(1, 2048 / (ti * tj));
  chunks = std::min<int64_t>(chunks, kChunksMax);
  chunks = std::min<int64_t>(chunks, std::max<int64_t>(1, rows / kRowsLds));
  int64_t per = (rows + chunks - 1) / chunks;
  per = (per + kRowsLds - 1) / kRowsLds * kRowsLds;
  chunks = (rows + per - 1) / per;
  MGM_CHECK((size_t)chunks * ka * kb <= part_cap, MGM_ERR_WORKSPACE, "block-product partial buffer too small");
  hipLaunchKernelGGL(k_ts_ahb, dim3((unsigned)(ti * tj), (unsigned)chunks), dim3(256), 0, c->stream, A, ka, B, kb,
                     rows, per, tj, part);
  const int64_t m = (int64_t)ka * kb;
  hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, c->stream, part, m, (int)chunks,
                     C);
  MGM_LAUNCH_CHECK();
}

size_t blk_part_entries(int ka_max, int kb_max) { return (size_t)kChunksMax * ka_max * kb_max; }

void blk_rowmul(Context* c, double2* W, int k, int64_t rows, const double2* M) {
  const int rows_pb = std::max(1, 2048 / k);
  const size_t lds = (size_t)rows_pb * k * sizeof(double2);
  MGM_CHECK(lds <= 65536, MGM_ERR_SHAPE, "block too wide for the row product");
  hipLaunchKernelGGL(k_rowmul, dim3((unsigned)((rows + rows_pb - 1) / rows_pb)), dim3(256), lds, c->stream, W, k,
                     rows, rows_pb, M);
  MGM_LAUNCH_CHECK();
}

void blk_gather(Context* c, const double2* W, int k, int c0, int b, int64_t nsite, int dof, bool g5, double2* out) {
  MGM_CHECK(c0 >= 0 && b >= 1 && c0 + b <= k, MGM_ERR_INVALID_ARG, "column range outside the block");
  hipLaunchKernelGGL(k_gather_cols, dim3(grid_of(nsite * dof * b)), dim3(256), 0, c->stream, W, k, c0, b, nsite, dof,
                     g5 ? 1 : 0, out);
  MGM_LAUNCH_CHECK();
}

void blk_scatter(Context* c, const double2* in, int k, int c0, int b, int64_t rows, double2* W) {
  MGM_CHECK(c0 >= 0 && b >= 1 && c0 + b <= k, MGM_ERR_INVALID_ARG, "column range outside the block");
  hipLaunchKernelGGL(k_scatter_cols, dim3(grid_of(rows * b)), dim3(256), 0, c->stream, in, k, c0, b, rows, W);
  MGM_LAUNCH_CHECK();
}

std::vector<std::complex<double>> blk_fetch(Context* c, const double2* C, size_t n) {
  std::vector<double2> h(n);
  MGM_HIP(hipMemcpyAsync(h.data(), C, sizeof(double2) * n, hipMemcpyDeviceToHost, c->stream));
  c->sync();
  std::vector<std::complex<double>> o(n);
  for (size_t i = 0; i < n; i++) o[i] = {h[i].x, h[i].y};
  return o;
}

void blk_cholqr(Context* c, double2* V, int k, int64_t rows, double2* part, size_t part_cap, double2* C, double2* M) {
  blk_ahb(c, V, k, V, k, rows, part, part_cap, C);
  using cd = std::complex<double>;
  std::vector<cd> G = blk_fetch(c, C, (size_t)k * k);
  std::vector<cd> R((size_t)k * k, 0.0), Ri((size_t)k * k, 0.0);
  // Cholesky G = R^H R, row by row of R
  for (int i = 0; i < k; i++) {
    MGM_CHECK(std::isfinite(G[(size_t)i * k + i].real()), MGM_ERR_NUMERIC, "non-finite Gram matrix");
    double d = G[(size_t)i * k + i].real();
    for (int p = 0; p < i; p++) d -= std::norm(R[(size_t)p * k + i]);
    MGM_CHECK(d > 1e-24 * G[(size_t)i * k + i].real() && d > 0, MGM_ERR_RANK_DEFICIENT,
              "block of vectors lost rank at column " + std::to_string(i));
    const double rii = std::sqrt(d);
    R[(size_t)i * k + i] = rii;
    for (int j = i + 1; j < k; j++) {
      cd s = G[(size_t)i * k + j];
      for (int p = 0; p < i; p++) s -= std::conj(R[(size_t)p * k + i]) * R[(size_t)p * k + j];
      R[(size_t)i * k + j] = s / rii;
    }
  }
  // Ri = R^-1 (upper triangular), column by column
  for (int j = 0; j < k; j++) {
    Ri[(size_t)j * k + j] = 1.0 / R[(size_t)j * k + j];
    for (int i = j - 1; i >= 0; i--) {
      cd s = 0.0;
      for (int p = i + 1; p <= j; p++) s += R[(size_t)i * k + p] * Ri[(size_t)p * k + j];
      Ri[(size_t)i * k + j] = -s / R[(size_t)i * k + i];
    }
  }
  std::vector<double2> hM((size_t)k * k);
  for (size_t e = 0; e < hM.size(); e++) hM[e] = make_double2(Ri[e].real(), Ri[e].imag());
  MGM_HIP(hipMemcpyAsync(M, hM.data(), sizeof(double2) * hM.size(), hipMemcpyHostToDevice, c->stream));
  blk_rowmul(c, V, k, rows, M);
  c->sync();  // hM leaves scope
}

}  // namespace mgm
