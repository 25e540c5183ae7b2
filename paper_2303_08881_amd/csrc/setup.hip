// setup.hip -- input validation, interface classification, interior-first
// permutation and extraction of the permuted subdomain blocks (Section 2.2.1,
// Fig. 1; Section 3.2, eq. (14)).  Integer work, bit-exact by construction.
#include "common.hpp"
#include "launch.hpp"

namespace silu {

// Validation of the CSR and the partition.  The first offending row (lowest
// index) is reported: the code goes through atomicCAS on a per-code basis and
// the row through atomicMin, so the result does not depend on scheduling.
__global__ void k_validate(const int64_t *rp, const int32_t *ci, int64_t n, int64_t nnz, const int32_t *part,
                           int32_t nparts, int32_t *err /* [0] csr-bad-row min, [1] part-bad-row min */) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t b = rp[i], e = rp[i + 1];
  bool bad = (i == 0 && b != 0) || (i == n - 1 && e != nnz) || e < b || b < 0 || e > nnz;
  if (!bad) {
    bool diag = false;
    int32_t prev = -1;
    for (int64_t p = b; p < e; p++) {
      const int32_t c = ci[p];
      if (c < 0 || c >= n || c <= prev) {
        bad = true;
        break;
      }
      prev = c;
      diag |= (c == i);
    }
    bad |= !diag;
  }
  if (bad) atomicMin(&err[0], (int32_t)i);
  if (part) {
    const int32_t p = part[i];
    if (p < 0 || p >= nparts) atomicMin(&err[1], (int32_t)i);
  }
}

int launch_validate(const int64_t *rp, const int32_t *ci, int64_t n, int64_t nnz, const int32_t *part,
                    int32_t nparts, void *err, hipStream_t s) {
  if (n == 0) return 0;
  k_validate<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rp, ci, n, nnz, part, nparts, (int32_t *)err);
  return check_launch("validate");
}

// Row i is interface when a_ij != 0 or a_ji != 0 for some j in another
// subdomain.  Every writer stores the same value 1, so the result is exact.
__global__ void k_classify(const int64_t *rp, const int32_t *ci, int64_t n, const int32_t *part, uint8_t *iface) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t pi = part ? part[i] : 0;
  bool mine = false;
  for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
    const int32_t j = ci[p];
    const int32_t pj = part ? part[j] : 0;
    if (pj != pi) {
      mine = true;
      iface[j] = 1;
    }
  }
  if (mine) iface[i] = 1;
}

int launch_classify(const int64_t *rp, const int32_t *ci, int64_t n, const int32_t *part, uint8_t *iface,
                    hipStream_t s) {
  if (n == 0) return 0;
  k_classify<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rp, ci, n, part, iface);
  return check_launch("classify");
}

// sort key: interior rows of subdomain p -> p, interface rows -> nparts + p
__global__ void k_perm_keys(int64_t n, const int32_t *part, int32_t nparts, const uint8_t *iface, uint32_t *key,
                            int32_t *val) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t p = part ? (uint32_t)part[i] : 0u;
  key[i] = iface[i] ? (uint32_t)nparts + p : p;
  val[i] = (int32_t)i;
}

int launch_perm_keys(int64_t n, const int32_t *part, int32_t nparts, const uint8_t *iface, uint32_t *key,
                     int32_t *val, hipStream_t s) {
  if (n == 0) return 0;
  k_perm_keys<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, part, nparts, iface, key, val);
  return check_launch("perm_keys");
}

__global__ void k_inverse_perm(int64_t n, const int32_t *perm, int32_t *iperm) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) iperm[perm[t]] = (int32_t)t;
}

int launch_inverse_perm(int64_t n, const int32_t *perm, int32_t *iperm, hipStream_t s) {
  if (n == 0) return 0;
  k_inverse_perm<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, perm, iperm);
  return check_launch("inverse_perm");
}

// counts of the permuted intra-subdomain block row and of the cross-subdomain
// coupling row (interface rows only) for each new row r
__global__ void k_extract_counts(const int64_t *rp, const int32_t *ci, int64_t n, int64_t nB, const int32_t *part,
                                 const int32_t *perm, int64_t *cnt_intra, int64_t *cnt_cross) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int32_t i = perm[r];
  const int32_t pi = part ? part[i] : 0;
  int64_t a = 0, c = 0;
  for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
    const int32_t j = ci[p];
    if ((part ? part[j] : 0) == pi)
      a++;
    else
      c++;
  }
  cnt_intra[r] = a;
  if (r >= nB) cnt_cross[r - nB] = c;
}

int launch_extract_counts(const int64_t *rp, const int32_t *ci, int64_t n, int64_t nB, const int32_t *part,
                          const int32_t *perm, int64_t *cnt_intra, int64_t *cnt_cross, hipStream_t s) {
  if (n == 0) return 0;
  k_extract_counts<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rp, ci, n, nB, part, perm, cnt_intra, cnt_cross);
  return check_launch("extract_counts");
}

// insertion sort of one row segment by column (rows are short; the order of
// equal keys cannot arise since columns are unique)
__device__ void sort_row(int32_t *c, double *v, int64_t m) {
  for (int64_t a = 1; a < m; a++) {
    const int32_t kc = c[a];
    const double kv = v[a];
    int64_t b = a - 1;
    while (b >= 0 && c[b] > kc) {
      c[b + 1] = c[b];
      v[b + 1] = v[b];
      b--;
    }
    c[b + 1] = kc;
    v[b + 1] = kv;
  }
}

__global__ void k_extract_fill(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, int64_t nB,
                               const int32_t *part, const int32_t *perm, const int32_t *iperm,
                               const int64_t *rp_intra, int32_t *ci_intra, double *v_intra, const int64_t *rp_cross,
                               int32_t *ci_cross, double *v_cross) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int32_t i = perm[r];
  const int32_t pi = part ? part[i] : 0;
  int64_t oa = rp_intra[r];
  int64_t oc = r >= nB ? rp_cross[r - nB] : 0;
  for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
    const int32_t j = ci[p];
    if ((part ? part[j] : 0) == pi) {
      ci_intra[oa] = iperm[j];
      v_intra[oa] = v[p];
      oa++;
    } else {
      ci_cross[oc] = (int32_t)(iperm[j] - nB);
      v_cross[oc] = v[p];
      oc++;
    }
  }
  sort_row(ci_intra + rp_intra[r], v_intra + rp_intra[r], rp_intra[r + 1] - rp_intra[r]);
  if (r >= nB) sort_row(ci_cross + rp_cross[r - nB], v_cross + rp_cross[r - nB], rp_cross[r - nB + 1] - rp_cross[r - nB]);
}

int launch_extract_fill(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, int64_t nB,
                        const int32_t *part, const int32_t *perm, const int32_t *iperm, const int64_t *rp_intra,
                        int32_t *ci_intra, double *v_intra, const int64_t *rp_cross, int32_t *ci_cross,
                        double *v_cross, hipStream_t s) {
  if (n == 0) return 0;
  k_extract_fill<<<(unsigned)((n + 127) / 128), 128, 0, s>>>(rp, ci, v, n, nB, part, perm, iperm, rp_intra, ci_intra,
                                                              v_intra, rp_cross, ci_cross, v_cross);
  return check_launch("extract_fill");
}

}  // namespace silu
