// Lowest eigenpairs of a graph Laplacian on the complement of its null space
// (the eigensolver of Section 6.4, in the form that section names as the
// alternative to FAS: the LAMG solver inside a block Rayleigh-quotient
// iteration, here LOBPCG (Knyazev 2001) with a few LAMG cycles as the
// preconditioner T ~ A^+).
//
// Blocks are n x k row-major in level 0's colour order (the solve's own
// layout), so the operator is the multi-vector residual kernel (b = 0) and the
// preconditioner the multi-vector cycle.  Per iteration:
//   R = A X - X Lambda;  W = T R, projected against X;  S = [X W P];
//   Rayleigh-Ritz on span(S): Gram matrices S^T S and S^T A S (q x q,
//   q <= 3 kb, FP64 partials per block, summed in a fixed order on the device),
//   small generalised eigenproblem on the host (column scaling, Jacobi
//   eigen-decomposition of the scaled S^T S with rank truncation, Jacobi on
//   the reduced S^T A S);
//   X <- S C,  P <- [W P] C_{W,P},  and the same combinations of A X, A W, A P,
//   so A is applied once per iteration (to W).
// The block carries kb = k + min(k, 4) columns (at most n / 4); the extra
// guard columns start from a counter-based hash and are not tested.
// Every block is kept zero-mean: the initial block is projected, T returns
// zero-mean corrections, and combinations of zero-mean blocks stay so.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "lamg_device.hpp"
#include "lamg_internal.hpp"
#include "../../include/lamg.h"

namespace lamg {
namespace {

constexpr int ET = 256;          // threads per block of the eigensolver kernels
constexpr int GRAM_ROWS = 32;    // rows of S and T staged in LDS per tile
constexpr int GRAM_BLOCKS = 1024; // fixed grid of the Gram kernel (fixes the sum order)
constexpr int EIG_MAX_K = 8;    // eigenpairs asked for
constexpr int EIG_MAX_KB = 16;  // iterated block: the asked pairs plus guard vectors
constexpr int QMAX = 3 * EIG_MAX_KB;
constexpr int CM_SLOTS = 8;     // coefficient slots of the combinations between synchronisations

struct Blocks3 {
  const double* p[3];
};

// part[i * q + j][b] = sum over the rows of block b's tiles of S[r, i] T[r, j],
// where column i of S is column i % k of block p[i / k] (likewise T); tiles
// are taken by blocks round-robin, rows in order inside a tile.  A thread's
// staging slots (LDS index e = r q + col) are fixed, so their source offsets
// are computed once, and the next tile is loaded into registers while the
// current one is reduced.
constexpr int GRAM_LPT = (GRAM_ROWS * QMAX + ET - 1) / ET;  // staging slots per thread
__device__ inline const double* pick(const Blocks3& B, int blk) {
  return blk == 0 ? B.p[0] : (blk == 1 ? B.p[1] : B.p[2]);
}
__global__ __launch_bounds__(ET) void k_gram(int n, int k, int nb, Blocks3 S, Blocks3 T, double* __restrict__ part) {
  __shared__ double sS[GRAM_ROWS * QMAX];
  __shared__ double sT[GRAM_ROWS * QMAX];
  const int q = nb * k, qq = q * q;
  const double* sp[GRAM_LPT];
  const double* tp[GRAM_LPT];
  int off[GRAM_LPT];
#pragma unroll
  for (int t = 0; t < GRAM_LPT; ++t) {
    const int e = threadIdx.x + t * ET;
    const int r = e / q, col = e % q, blk = min(col / k, nb - 1), c = col % k;
    off[t] = r * k + c;
    sp[t] = pick(S, blk);
    tp[t] = pick(T, blk);
  }
  // running sums, one slot per (i, j), each owned by one thread
  __shared__ double sAcc[QMAX * QMAX];
  for (int pij = threadIdx.x; pij < qq; pij += ET) sAcc[pij] = 0.0;
  const int ntiles = (n + GRAM_ROWS - 1) / GRAM_ROWS;
  double ps[GRAM_LPT], pt[GRAM_LPT];
  int tile = blockIdx.x;
  if (tile < ntiles) {
    const int r0 = tile * GRAM_ROWS, lim = min(GRAM_ROWS, n - r0) * q;
    const size_t base = (size_t)r0 * k;
#pragma unroll
    for (int t = 0; t < GRAM_LPT; ++t)
      if ((int)threadIdx.x + t * ET < lim) {
        ps[t] = sp[t][base + off[t]];
        pt[t] = tp[t][base + off[t]];
      }
  }
  for (; tile < ntiles; tile += gridDim.x) {
    const int rows = min(GRAM_ROWS, n - tile * GRAM_ROWS);
#pragma unroll
    for (int t = 0; t < GRAM_LPT; ++t) {
      const int e = threadIdx.x + t * ET;
      if (e < rows * q) {
        sS[e] = ps[t];
        sT[e] = pt[t];
      }
    }
    __syncthreads();
    const int nt = tile + gridDim.x;
    if (nt < ntiles) {
      const int r0 = nt * GRAM_ROWS, lim = min(GRAM_ROWS, n - r0) * q;
      const size_t base = (size_t)r0 * k;
#pragma unroll
      for (int t = 0; t < GRAM_LPT; ++t)
        if ((int)threadIdx.x + t * ET < lim) {
          ps[t] = sp[t][base + off[t]];
          pt[t] = tp[t][base + off[t]];
        }
    }
#pragma unroll 1
    for (int pij = threadIdx.x; pij < qq; pij += ET) {
      const int i = pij / q, j = pij % q;
      double a = sAcc[pij];
      int r = 0;
      // eight rows' operands in flight, then their products in row order
      for (; r + 8 <= rows; r += 8) {
        double xv[8], yv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          xv[u] = sS[(r + u) * q + i];
          yv[u] = sT[(r + u) * q + j];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) a += xv[u] * yv[u];
      }
      for (; r < rows; ++r) a += sS[r * q + i] * sT[r * q + j];
      sAcc[pij] = a;
    }
    __syncthreads();
  }
  for (int pij = threadIdx.x; pij < qq; pij += ET) part[(size_t)pij * gridDim.x + blockIdx.x] = sAcc[pij];
}

// g[p] = sum over blocks b of part[p][b]: one workgroup per entry, each
// thread sums a strided slice in order, then a fixed pairwise tree in LDS
__global__ __launch_bounds__(ET) void k_gram_finish(int nblk, const double* __restrict__ part, double* __restrict__ g) {
  __shared__ double red[ET];
  const int p = blockIdx.x;
  const double* row = part + (size_t)p * nblk;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += ET) s += row[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = ET / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) g[p] = red[0];
}

// out[r, c] = sum_{i < nb k} Src[r, i] C[i, c]  (C is q x k row-major; the
// sum runs over the source columns in order).  One thread per row: the row
// is read once, C at wave-uniform addresses.
__global__ __launch_bounds__(ET) void k_combine(int n, int k, int nb, Blocks3 S, const double* __restrict__ Cm,
                                                double* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double acc[EIG_MAX_KB];
#pragma unroll
  for (int c = 0; c < EIG_MAX_KB; ++c) acc[c] = 0.0;
  for (int blk = 0; blk < nb; ++blk) {
    const double* row = S.p[blk] + (size_t)r * k;
    for (int i = 0; i < k; ++i) {
      const double v = row[i];
      const double* crow = Cm + (blk * k + i) * k;
#pragma unroll
      for (int c = 0; c < EIG_MAX_KB; ++c)
        if (c < k) acc[c] += v * crow[c];
    }
  }
  double* o = out + (size_t)r * k;
#pragma unroll
  for (int c = 0; c < EIG_MAX_KB; ++c)
    if (c < k) o[c] = acc[c];
}

// splitmix64 (Vigna): a counter-based generator, mapped to [-1, 1)
__device__ inline double guard_value(uint64_t ctr) {
  uint64_t z = ctr + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

// Initial n x kb block in colour order: out[i, c] = B[perm[i], c] for the k
// given columns, a hash of (perm[i], c) for the guard columns c >= k.
__global__ void k_eig_init(int n, int k, int kb, const int* __restrict__ perm, const double* __restrict__ B,
                           double* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)n * kb) return;
  const int i = (int)(g / kb), c = (int)(g % kb);
  const int u = perm[i];
  out[g] = c < k ? B[(size_t)u * k + c] : guard_value((uint64_t)u * EIG_MAX_KB + (uint64_t)c);
}
// out[perm[i], c] = a[i, c] for the first k of kb columns
__global__ void k_eig_scatter(int n, int k, int kb, const int* __restrict__ perm, const double* __restrict__ a,
                              double* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)n * k) return;
  const int i = (int)(g / k), c = (int)(g % k);
  out[(size_t)perm[i] * k + c] = a[(size_t)i * kb + c];
}

inline dim3 grid_nk(int64_t nk) { return dim3((unsigned)std::max<int64_t>(1, (nk + ET - 1) / ET)); }

// Cyclic Jacobi eigen-decomposition of a symmetric q x q matrix (row-major):
// w receives the eigenvalues ascending and v the
// eigenvectors as columns (v[i * q + j] = component i of vector j).
void jacobi_eig(int q, std::vector<double> a, std::vector<double>& w, std::vector<double>& v) {
  std::vector<double> V((size_t)q * q, 0.0);
  for (int i = 0; i < q; ++i) V[(size_t)i * q + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j) {
        const double x = a[(size_t)i * q + j] * a[(size_t)i * q + j];
        tot += x;
        if (i != j) off += x;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < q; ++p)
      for (int r = p + 1; r < q; ++r) {
        const double apr = a[(size_t)p * q + r];
        if (apr == 0.0) continue;
        const double app = a[(size_t)p * q + p], arr = a[(size_t)r * q + r];
        // rotation that zeroes a_pr (Golub and Van Loan, symmetric Schur 2x2)
        const double tau = (arr - app) / (2.0 * apr);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int i = 0; i < q; ++i) {
          const double aip = a[(size_t)i * q + p], air = a[(size_t)i * q + r];
          a[(size_t)i * q + p] = c * aip - s * air;
          a[(size_t)i * q + r] = s * aip + c * air;
        }
        for (int i = 0; i < q; ++i) {
          const double api = a[(size_t)p * q + i], ari = a[(size_t)r * q + i];
          a[(size_t)p * q + i] = c * api - s * ari;
          a[(size_t)r * q + i] = s * api + c * ari;
        }
        for (int i = 0; i < q; ++i) {
          const double vip = V[(size_t)i * q + p], vir = V[(size_t)i * q + r];
          V[(size_t)i * q + p] = c * vip - s * vir;
          V[(size_t)i * q + r] = s * vip + c * vir;
        }
      }
  }
  std::vector<int> ord(q);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return a[(size_t)x * q + x] < a[(size_t)y * q + y]; });
  w.assign(q, 0.0);
  v.assign((size_t)q * q, 0.0);
  for (int j = 0; j < q; ++j) {
    w[j] = a[(size_t)ord[j] * q + ord[j]];
    for (int i = 0; i < q; ++i) v[(size_t)i * q + j] = V[(size_t)i * q + ord[j]];
  }
}

// Rayleigh-Ritz on span(S): GB = S^T S, GA = S^T A S (q x q).  Returns the
// number of kept directions (>= k on success) and fills C (q x k) with the
// coefficients of the k lowest Ritz vectors (C^T GB C = I) and theta.
int rayleigh_ritz(int q, int k, const std::vector<double>& GB, const std::vector<double>& GA,
                  std::vector<double>& Cm, std::vector<double>& theta) {
  std::vector<double> d(q);
  for (int i = 0; i < q; ++i) {
    const double g = GB[(size_t)i * q + i];
    if (!(g > 0.0) || !std::isfinite(g)) return 0;
    d[i] = 1.0 / std::sqrt(g);
  }
  std::vector<double> b((size_t)q * q), a((size_t)q * q);
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) {
      b[(size_t)i * q + j] = 0.5 * (GB[(size_t)i * q + j] + GB[(size_t)j * q + i]) * d[i] * d[j];
      a[(size_t)i * q + j] = 0.5 * (GA[(size_t)i * q + j] + GA[(size_t)j * q + i]) * d[i] * d[j];
    }
  std::vector<double> wb, vb;
  jacobi_eig(q, b, wb, vb);
  const double top = wb[q - 1];
  std::vector<int> keep;
  for (int j = 0; j < q; ++j)
    if (wb[j] > 1e-10 * top) keep.push_back(j);
  const int r = (int)keep.size();
  if (r < k) return r;
  // basis Z = D Vb_keep Wb_keep^-1/2 (q x r); reduced matrix Z^T GA Z (D applied above)
  std::vector<double> Z((size_t)q * r);
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < r; ++j) Z[(size_t)i * r + j] = vb[(size_t)i * q + keep[j]] / std::sqrt(wb[keep[j]]);
  std::vector<double> AZ((size_t)q * r, 0.0), red((size_t)r * r, 0.0);
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < r; ++j) {
      double s = 0.0;
      for (int t = 0; t < q; ++t) s += a[(size_t)i * q + t] * Z[(size_t)t * r + j];
      AZ[(size_t)i * r + j] = s;
    }
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      double s = 0.0;
      for (int t = 0; t < q; ++t) s += Z[(size_t)t * r + i] * AZ[(size_t)t * r + j];
      red[(size_t)i * r + j] = s;
    }
  for (int i = 0; i < r; ++i)
    for (int j = i + 1; j < r; ++j) {
      const double m = 0.5 * (red[(size_t)i * r + j] + red[(size_t)j * r + i]);
      red[(size_t)i * r + j] = red[(size_t)j * r + i] = m;
    }
  std::vector<double> wa, va;
  jacobi_eig(r, red, wa, va);
  Cm.assign((size_t)q * k, 0.0);
  theta.assign(wa.begin(), wa.begin() + k);
  for (int i = 0; i < q; ++i)
    for (int c = 0; c < k; ++c) {
      double s = 0.0;
      for (int j = 0; j < r; ++j) s += Z[(size_t)i * r + j] * va[(size_t)j * r + c];
      Cm[(size_t)i * k + c] = d[i] * s;
    }
  return r;
}

struct EigWork {
  Hierarchy* H;
  int n, k;
  std::vector<void*> owned;
  double* part = nullptr;
  double* g = nullptr;   // device q*q
  double* cm = nullptr;   // device CM_SLOTS x (QMAX * k) coefficient slots
  double* hcm = nullptr;  // pinned host staging of the same slots
  double* hg = nullptr;   // pinned host mirror of g
  int slot = 0;           // next free coefficient slot; all are free after a synchronisation
  double* blk(size_t nk) {
    void* p = dev_alloc(H->o, nk * sizeof(double) + 16);
    owned.push_back(p);
    return (double*)p;
  }
  ~EigWork() {
    (void)hipStreamSynchronize(H->s);  // combinations may still be in flight on an early return
    for (void* p : owned) dev_free(H->o, p);
    if (hg) (void)hipHostFree(hg);
    if (hcm) (void)hipHostFree(hcm);
  }
  // host q x q matrix S^T T
  std::vector<double> gram(int nb, Blocks3 S, Blocks3 T) {
    const int q = nb * k, qq = q * q;
    hipStream_t s = H->s;
    hipLaunchKernelGGL(k_gram, dim3(GRAM_BLOCKS), dim3(ET), 0, s, n, k, nb, S, T, part);
    hipLaunchKernelGGL(k_gram_finish, dim3(qq), dim3(ET), 0, s, GRAM_BLOCKS, (const double*)part, g);
    LAMG_HIP(hipMemcpyAsync(hg, g, (size_t)qq * sizeof(double), hipMemcpyDeviceToHost, s));
    LAMG_HIP(hipStreamSynchronize(s));
    slot = 0;
    return std::vector<double>(hg, hg + qq);
  }
  void combine(int nb, Blocks3 S, const std::vector<double>& C, int row0, double* out) {
    // rows row0 .. row0 + nb k of C (q_total x k) as the coefficient matrix
    // Each combination takes its own coefficient slot, so none waits for the
    // previous one; the slots are recycled after a synchronisation.
    hipStream_t s = H->s;
    if (slot == CM_SLOTS) {
      LAMG_HIP(hipStreamSynchronize(s));
      slot = 0;
    }
    const size_t cnt = (size_t)nb * k * k, o = (size_t)slot * QMAX * k;
    std::copy(C.begin() + (size_t)row0 * k, C.begin() + (size_t)row0 * k + cnt, hcm + o);
    LAMG_HIP(hipMemcpyAsync(cm + o, hcm + o, cnt * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_combine, grid_nk(n), dim3(ET), 0, s, n, k, nb, S, (const double*)(cm + o), out);
    LAMG_HIP(hipGetLastError());
    ++slot;
  }
};

}  // namespace

lamg_status eigs(Hierarchy* H, int k, double* X, double* evals, double tol, int max_iter, int cycles,
                 int32_t* iters, double* resid) {
  const int n = H->lv[0].n;
  if (k < 1 || k > EIG_MAX_K || 4 * k > n || max_iter < 0 || cycles < 1 || !(tol > 0.0)) return LAMG_E_INVALID_ARG;
  // guard vectors: the last pairs of a block converge at the rate set by the
  // gap to the first eigenvalue outside it, so the block carries extra
  // columns and only the first k are tested
  const int kb = std::max(k, std::min(k + std::min(k, 4), n / 4));
  hipStream_t s = H->s;
  const int64_t nk = (int64_t)n * kb;
  EigWork E;
  E.H = H;
  E.n = n;
  E.k = kb;
  E.part = E.blk((size_t)GRAM_BLOCKS * QMAX * QMAX);
  E.g = E.blk((size_t)QMAX * QMAX);
  E.cm = E.blk((size_t)CM_SLOTS * QMAX * kb);
  LAMG_HIP(hipHostMalloc((void**)&E.hcm, (size_t)CM_SLOTS * QMAX * kb * sizeof(double), hipHostMallocDefault));
  LAMG_HIP(hipHostMalloc((void**)&E.hg, (size_t)QMAX * QMAX * sizeof(double), hipHostMallocDefault));
  double *Xb = E.blk(nk), *NX = E.blk(nk), *Wb = E.blk(nk), *NW = E.blk(nk), *Pb = E.blk(nk), *NP = E.blk(nk);
  double *R = E.blk(nk), *Xn = E.blk(nk), *NXn = E.blk(nk), *Pn = E.blk(nk), *NPn = E.blk(nk);
  const int* perm = H->lv[0].perm;

  hipLaunchKernelGGL(k_eig_init, grid_nk(nk), dim3(ET), 0, s, n, k, kb, perm, (const double*)X, Xb);
  mv_project(H, kb, Xb);
  mv_neg_apply(H, kb, Xb, NX);
  std::vector<double> C, theta;
  // Rayleigh-Ritz on span(X) alone: orthonormal X, Ritz values in theta
  auto rr_x = [&]() {
    const std::vector<double> GB = E.gram(1, Blocks3{{Xb, nullptr, nullptr}}, Blocks3{{Xb, nullptr, nullptr}});
    std::vector<double> GA = E.gram(1, Blocks3{{Xb, nullptr, nullptr}}, Blocks3{{NX, nullptr, nullptr}});
    for (double& v : GA) v = -v;
    if (rayleigh_ritz(kb, kb, GB, GA, C, theta) < kb) return false;
    E.combine(1, Blocks3{{Xb, nullptr, nullptr}}, C, 0, Xn);
    E.combine(1, Blocks3{{NX, nullptr, nullptr}}, C, 0, NXn);
    std::swap(Xb, Xn);
    std::swap(NX, NXn);
    return true;
  };
  int it = 0;
  auto breakdown = [&]() {
    if (iters) *iters = it;  // X and evals untouched
    return LAMG_E_BREAKDOWN;
  };
  if (!rr_x()) return breakdown();
  bool haveP = false;
  std::vector<double> rn(kb, 0.0);
  // R = A X - X Lambda = -(NX) - X Lambda and its column norms in rn; false
  // if a norm or a Ritz value is not finite
  auto residuals = [&]() {
    std::vector<double> Cr((size_t)2 * kb * kb, 0.0);
    for (int c = 0; c < kb; ++c) {
      Cr[(size_t)c * kb + c] = -1.0;
      Cr[(size_t)(kb + c) * kb + c] = -theta[c];
    }
    E.combine(2, Blocks3{{NX, Xb, nullptr}}, Cr, 0, R);
    const std::vector<double> GR = E.gram(1, Blocks3{{R, nullptr, nullptr}}, Blocks3{{R, nullptr, nullptr}});
    bool ok = true;
    for (int c = 0; c < kb; ++c) {
      rn[c] = std::sqrt(std::max(0.0, GR[(size_t)c * kb + c]));
      if (!std::isfinite(rn[c]) || !std::isfinite(theta[c])) ok = false;
    }
    return ok;
  };
  lamg_status st = LAMG_E_NOT_CONVERGED;
  for (;;) {
    if (!residuals()) return breakdown();
    bool done = true;
    for (int c = 0; c < k; ++c)
      if (rn[c] > tol * std::fabs(theta[c])) done = false;
    if (done) { st = LAMG_OK; break; }
    if (it >= max_iter) break;
    ++it;
    mv_precondition(H, kb, R, Wb, cycles);
    // W <- W - X (X^T W), twice: with T ~ A^+ the new directions lie close to
    // span(X), and without this the Gram matrices of [X W P] are too
    // ill-conditioned for the residual to fall below ~1e-7 relative.  A is
    // applied to the projected W, so A W carries no cancellation error.
    for (int pass = 0; pass < 2; ++pass) {
      const std::vector<double> XW = E.gram(1, Blocks3{{Xb, nullptr, nullptr}}, Blocks3{{Wb, nullptr, nullptr}});
      std::vector<double> Cp((size_t)2 * kb * kb, 0.0);
      for (int i = 0; i < kb; ++i) {
        Cp[(size_t)i * kb + i] = 1.0;
        for (int c = 0; c < kb; ++c) Cp[(size_t)(kb + i) * kb + c] = -XW[(size_t)i * kb + c];
      }
      E.combine(2, Blocks3{{Wb, Xb, nullptr}}, Cp, 0, Xn);
      std::swap(Wb, Xn);
    }
    mv_neg_apply(H, kb, Wb, NW);
    int nb = haveP ? 3 : 2;
    for (;;) {
      const Blocks3 S{{Xb, Wb, nb == 3 ? Pb : nullptr}}, NS{{NX, NW, nb == 3 ? NP : nullptr}};
      const std::vector<double> GB = E.gram(nb, S, S);
      std::vector<double> GA = E.gram(nb, S, NS);
      for (double& v : GA) v = -v;
      const int r = rayleigh_ritz(nb * kb, kb, GB, GA, C, theta);
      if (r >= kb) break;
      if (nb == 2) return breakdown();
      nb = 2;  // drop the search directions and retry
    }
    const Blocks3 S{{Xb, Wb, nb == 3 ? Pb : nullptr}}, NS{{NX, NW, nb == 3 ? NP : nullptr}};
    const Blocks3 SP{{Wb, nb == 3 ? Pb : nullptr, nullptr}}, NSP{{NW, nb == 3 ? NP : nullptr, nullptr}};
    E.combine(nb, S, C, 0, Xn);
    E.combine(nb, NS, C, 0, NXn);
    E.combine(nb - 1, SP, C, kb, Pn);
    E.combine(nb - 1, NSP, C, kb, NPn);
    std::swap(Xb, Xn);
    std::swap(NX, NXn);
    std::swap(Pb, Pn);
    std::swap(NP, NPn);
    haveP = true;
  }
  // a last Rayleigh-Ritz on the final block restores orthonormality lost to
  // the ill-conditioned Gram matrices of the last iterations; the residuals
  // returned are those of the block it produces
  if (!rr_x() || !residuals()) return breakdown();
  hipLaunchKernelGGL(k_eig_scatter, grid_nk((int64_t)n * k), dim3(ET), 0, s, n, k, kb, perm, (const double*)Xb, X);
  LAMG_HIP(hipGetLastError());
  LAMG_HIP(hipStreamSynchronize(s));
  for (int c = 0; c < k; ++c) {
    evals[c] = theta[c];
    if (resid) resid[c] = theta[c] != 0.0 ? rn[c] / std::fabs(theta[c]) : rn[c];
  }
  if (iters) *iters = it;
  return st;
}

}  // namespace lamg

using namespace lamg;

extern "C" {

lamg_status lamg_eigs(lamg_handle h, int32_t k, double* X, double* evals, double tol, int32_t max_iter,
                      int32_t cycles, int32_t* iters, double* resid) {
  if (!h || !X || !evals) return LAMG_E_INVALID_ARG;
  roctxRangePushA("lamg_eigs");
  struct Pop {
    ~Pop() { roctxRangePop(); }
  } pop;
  try {
    return eigs(&h->H, k, X, evals, tol, max_iter, cycles, iters, resid);
  } catch (const DevError& e) {
    set_last_error("lamg_eigs", e.e);
    return e.e == hipErrorOutOfMemory ? LAMG_E_OUT_OF_MEMORY : LAMG_E_DEVICE;
  }
}

}  // extern "C"
