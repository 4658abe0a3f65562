// Box tables, interaction lists, near-field lists and needed slots on the
// device (Section 2.2; the slot closure follows the data flow of Algorithm 1).
//
// From the Morton-sorted point keys: per level l the non-empty boxes are the
// segment heads of key >> 3(D - l), with their point ranges, integer
// coordinates, parents and child ranges.  Per level l >= 1 the interaction
// list I^B holds the non-empty children of the boxes of N^{parent(B)} that are
// not in N^B, as pairs (B, A) sorted by (B, A), with the wedge of A seen from B
// (l_in = dir(n)) and of B seen from A (l_out = dir(-n)), n = i_A - i_B.  The
// near-field list of a leaf holds its adjacent leaves (itself included) in
// increasing order.  A (box, wedge) slot is needed when a pair uses it or when
// the parent's slot of the wedge containing it is needed (M2M reads the
// children, L2L writes them).  The tests are the integer forms of geometry.hpp.
// Every table is copied back to the host, where the translation tables are
// built from it.
#include <hip/hip_runtime.h>


#include <algorithm>
#include <vector>

#include "geometry.hpp"
#include "internal.hpp"

namespace dfmm {

namespace {

constexpr int kBS = 256;

unsigned nblk(int64_t n) { return unsigned(std::max<int64_t>(1, (n + kBS - 1) / kBS)); }

__device__ __forceinline__ int64_t d_morton(int64_t x, int64_t y, int64_t z, int bits) {
  int64_t k = 0;
  for (int b = 0; b < bits; ++b)
    k |= (((x >> b) & 1) << (3 * b)) | (((y >> b) & 1) << (3 * b + 1)) | (((z >> b) & 1) << (3 * b + 2));
  return k;
}

// index of the box with Morton key k among the nb ascending keys, or -1
__device__ __forceinline__ int d_find(const int64_t* __restrict__ keys, int nb, int64_t k) {
  int lo = 0, hi = nb;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (keys[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return (lo < nb && keys[lo] == k) ? lo : -1;
}

__global__ void k_heads(const unsigned long long* __restrict__ key, int64_t n, unsigned sh, int* __restrict__ head) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= n) return;
  head[s] = (s == 0 || (key[s] >> sh) != (key[s - 1] >> sh)) ? 1 : 0;
}

// box b of a level starts at the point s where the inclusive head count reaches b + 1
__global__ void k_boxes(const unsigned long long* __restrict__ key, int64_t n, unsigned sh, int l,
                        const int* __restrict__ head, const int* __restrict__ incl, int64_t* __restrict__ bkey,
                        int* __restrict__ bstart, int* __restrict__ cx, int* __restrict__ cy, int* __restrict__ cz) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= n || !head[s]) return;
  const int b = incl[s] - 1;
  const int64_t k = int64_t(key[s] >> sh);
  bkey[b] = k;
  bstart[b] = int(s);
  int c[3] = {0, 0, 0};
  for (int i = 0; i < l; ++i)
    for (int a = 0; a < 3; ++a) c[a] |= int((k >> (3 * i + a)) & 1) << i;
  cx[b] = c[0];
  cy[b] = c[1];
  cz[b] = c[2];
}

__global__ void k_box_end(const int* __restrict__ bstart, int nb, int n, int* __restrict__ bend) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  bend[b] = b + 1 < nb ? bstart[b + 1] : n;
}

// parent of each box: the parent-level box of its first point
__global__ void k_parent(const int* __restrict__ bstart, int nb, const int* __restrict__ incl_up,
                         int* __restrict__ parent) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  parent[b] = incl_up[bstart[b]] - 1;
}

// child range of each box: the child-level boxes of its first and last point
__global__ void k_children(const int* __restrict__ bstart, const int* __restrict__ bend, int nb,
                           const int* __restrict__ incl_dn, int* __restrict__ cbeg, int* __restrict__ cend) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  cbeg[b] = incl_dn[bstart[b]] - 1;
  cend[b] = incl_dn[bend[b] - 1];
}

struct LvView {  // device box table of one level
  const int64_t* key;
  const int *cx, *cy, *cz, *parent, *cbeg, *cend;
  int nb, l;
};

// I^B of every box B of level l (EMIT = 0: count, 1: write (B, A) keys)
template <int EMIT>
__global__ void k_pairs(LvView L, LvView U, int e2, const int* __restrict__ noff, int nnoff,
                        int* __restrict__ cnt, const int* __restrict__ off, unsigned long long* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= L.nb) return;
  const int p = L.parent[b];
  const int64_t side = int64_t(1) << U.l;
  int k = 0;
  const int o = EMIT ? off[b] : 0;
  for (int i = 0; i < nnoff; ++i) {
    const int64_t qx = U.cx[p] + noff[3 * i], qy = U.cy[p] + noff[3 * i + 1], qz = U.cz[p] + noff[3 * i + 2];
    if (qx < 0 || qy < 0 || qz < 0 || qx >= side || qy >= side || qz >= side) continue;
    const int q = d_find(U.key, U.nb, d_morton(qx, qy, qz, U.l));
    if (q < 0) continue;
    for (int a = U.cbeg[q]; a < U.cend[q]; ++a) {
      if (is_near_e2(L.cx[a] - L.cx[b], L.cy[a] - L.cy[b], L.cz[a] - L.cz[b], e2)) continue;
      if (EMIT) out[o + k] = (static_cast<unsigned long long>(b) << 32) | static_cast<unsigned>(a);
      ++k;
    }
  }
  if (!EMIT) cnt[b] = k;
}

__global__ void k_pair_fields(const unsigned long long* __restrict__ key, int64_t np, LvView L, int e2,
                              int* __restrict__ out) {  // out: [np][7] (B, A, nx, ny, nz, din, dout)
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const int b = int(key[i] >> 32), a = int(key[i] & 0xffffffffu);
  const int nx = L.cx[a] - L.cx[b], ny = L.cy[a] - L.cy[b], nz = L.cz[a] - L.cz[b];
  int din = -1, dout = -1;
  if (e2 >= 1) {
    const int64_t w = int64_t(1) << (e2 - 1);
    din = direction(nx, ny, nz, w);
    dout = direction(-nx, -ny, -nz, w);
  }
  int* r = out + 7 * i;
  r[0] = b;
  r[1] = a;
  r[2] = nx;
  r[3] = ny;
  r[4] = nz;
  r[5] = din;
  r[6] = dout;
}

// adjacent leaves of each leaf, ascending (EMIT = 0: count)
template <int EMIT>
__global__ void k_near(LvView L, const int* __restrict__ noff, int nnoff, int* __restrict__ cnt,
                       const int* __restrict__ off, int* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= L.nb) return;
  const int64_t side = int64_t(1) << L.l;
  int v[27];
  int k = 0;
  for (int i = 0; i < nnoff && k < 27; ++i) {
    const int64_t x = L.cx[b] + noff[3 * i], y = L.cy[b] + noff[3 * i + 1], z = L.cz[b] + noff[3 * i + 2];
    if (x < 0 || y < 0 || z < 0 || x >= side || y >= side || z >= side) continue;
    const int a = d_find(L.key, L.nb, d_morton(x, y, z, L.l));
    if (a >= 0) v[k++] = a;
  }
  if (!EMIT) {
    cnt[b] = k;
    return;
  }
  for (int i = 1; i < k; ++i) {  // insertion sort (k <= 27)
    const int x = v[i];
    int j = i - 1;
    while (j >= 0 && v[j] > x) {
      v[j + 1] = v[j];
      --j;
    }
    v[j + 1] = x;
  }
  for (int i = 0; i < k; ++i) out[off[b] + i] = v[i];
}

__global__ void k_mark_pairs(const int* __restrict__ f, int64_t np, int ndir, int* __restrict__ out_f,
                             int* __restrict__ in_f) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const int* r = f + 7 * i;
  out_f[int64_t(r[1]) * ndir + r[6]] = 1;  // (A, l_out)
  in_f[int64_t(r[0]) * ndir + r[5]] = 1;   // (B, l_in)
}

// needed slots of the parent level pass to the children (wedge l -> l down)
__global__ void k_mark_down(const int* __restrict__ pout, const int* __restrict__ pin, int npb, int ndir_p,
                            int64_t w2, const int* __restrict__ cbeg, const int* __restrict__ cend, int ndir,
                            int* __restrict__ out_f, int* __restrict__ in_f) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(npb) * ndir_p) return;
  const int p = int(t / ndir_p), d = int(t % ndir_p);
  const int dd = direction_down(d, w2);
  for (int c = cbeg[p]; c < cend[p]; ++c) {
    if (pout[t]) out_f[int64_t(c) * ndir + dd] = 1;
    if (pin[t]) in_f[int64_t(c) * ndir + dd] = 1;
  }
}

template <class T>
std::vector<T> download(const DevBuf& b, int64_t n) {
  std::vector<T> h(size_t(std::max<int64_t>(0, n)));
  if (n > 0) DFMM_HIP(hipMemcpy(h.data(), b.p, sizeof(T) * size_t(n), hipMemcpyDeviceToHost));
  return h;
}

int64_t last_int(const DevBuf& b, int64_t i) {
  int v = 0;
  DFMM_HIP(hipMemcpy(&v, static_cast<const int*>(b.p) + i, sizeof(int), hipMemcpyDeviceToHost));
  return v;
}

// counts -> exclusive offsets (device) and the total
int64_t offsets_of(const DevBuf& cnt, DevBuf& off, int64_t n) {
  off.alloc(sizeof(int) * size_t(n + 1));
  if (n == 0) return 0;
  scan_excl(cnt.as<int>(), off.as<int>(), n);
  const int64_t tot = last_int(off, n - 1) + last_int(cnt, n - 1);
  if (tot > (int64_t(1) << 31) - 1) throw Error{DFMM_EUNSUPPORTED, "list larger than 2^31 entries"};
  return tot;
}

// offset table (x, y, z triples) on the device; returns the number of offsets
int upload_offsets(const std::vector<int64_t>& noff, DevBuf& d) {
  std::vector<int32_t> v(noff.begin(), noff.end());
  d.upload(v);
  return int(v.size() / 3);
}

LvView view_of(const DevTree& DT, int l) {
  const DevLevel& L = DT.lv[size_t(l)];
  return LvView{L.key.as<int64_t>(), L.cx.as<int>(), L.cy.as<int>(), L.cz.as<int>(), L.parent.as<int>(),
                L.cbeg.as<int>(), L.cend.as<int>(), int(L.nb), l};
}

}  // namespace

void build_levels_device(const unsigned long long* key, int64_t N, int D, Tree& T, DevTree& DT) {
  if (N > (int64_t(1) << 31) - 1) throw Error{DFMM_EINVAL, "too many points"};
  DT.lv.clear();
  DT.lv.resize(size_t(D) + 1);
  DT.incl.clear();
  DT.incl.resize(size_t(D) + 1);
  DevBuf head;
  head.alloc(sizeof(int) * size_t(N));
  for (int l = 0; l <= D; ++l) {
    const unsigned sh = unsigned(3 * (D - l));
    DevLevel& L = DT.lv[size_t(l)];
    DevBuf& incl = DT.incl[size_t(l)];
    incl.alloc(sizeof(int) * size_t(N));
    hipLaunchKernelGGL(k_heads, dim3(nblk(N)), dim3(kBS), 0, 0, key, N, sh, head.as<int>());
    scan_incl(head.as<int>(), incl.as<int>(), N);
    L.nb = last_int(incl, N - 1);
    const size_t nb = size_t(L.nb);
    L.key.alloc(sizeof(int64_t) * nb);
    for (DevBuf* b : {&L.start, &L.end, &L.cx, &L.cy, &L.cz, &L.parent, &L.cbeg, &L.cend}) b->alloc(sizeof(int) * nb);
    hipLaunchKernelGGL(k_boxes, dim3(nblk(N)), dim3(kBS), 0, 0, key, N, sh, l, head.as<int>(), incl.as<int>(),
                       L.key.as<int64_t>(), L.start.as<int>(), L.cx.as<int>(), L.cy.as<int>(), L.cz.as<int>());
    hipLaunchKernelGGL(k_box_end, dim3(nblk(L.nb)), dim3(kBS), 0, 0, L.start.as<int>(), int(L.nb), int(N),
                       L.end.as<int>());
    if (l > 0)
      hipLaunchKernelGGL(k_parent, dim3(nblk(L.nb)), dim3(kBS), 0, 0, L.start.as<int>(), int(L.nb),
                         DT.incl[size_t(l) - 1].as<int>(), L.parent.as<int>());
    else
      DFMM_HIP(hipMemset(L.parent.p, 0xff, sizeof(int) * nb));
  }
  for (int l = 0; l <= D; ++l) {
    DevLevel& L = DT.lv[size_t(l)];
    if (l < D)
      hipLaunchKernelGGL(k_children, dim3(nblk(L.nb)), dim3(kBS), 0, 0, L.start.as<int>(), L.end.as<int>(),
                         int(L.nb), DT.incl[size_t(l) + 1].as<int>(), L.cbeg.as<int>(), L.cend.as<int>());
    else {
      DFMM_HIP(hipMemset(L.cbeg.p, 0, sizeof(int) * size_t(L.nb)));
      DFMM_HIP(hipMemset(L.cend.p, 0, sizeof(int) * size_t(L.nb)));
    }
  }
  DFMM_HIP(hipGetLastError());
  // host copies
  T.lv.assign(size_t(D) + 1, {});
  for (int l = 0; l <= D; ++l) {
    const DevLevel& L = DT.lv[size_t(l)];
    Tree::Lv& H = T.lv[size_t(l)];
    const int64_t nb = L.nb;
    H.key = download<int64_t>(L.key, nb);
    auto cp = [&](const DevBuf& b, std::vector<int64_t>& dst) {
      std::vector<int> v = download<int>(b, nb);
      dst.assign(v.begin(), v.end());
    };
    cp(L.cx, H.cx);
    cp(L.cy, H.cy);
    cp(L.cz, H.cz);
    cp(L.start, H.start);
    cp(L.end, H.end);
    cp(L.parent, H.parent);
    H.octant.resize(size_t(nb));
    for (int64_t b = 0; b < nb; ++b) H.octant[size_t(b)] = l > 0 ? (H.key[size_t(b)] & 7) : 0;
    if (l < D) {
      cp(L.cbeg, H.cbeg);
      cp(L.cend, H.cend);
    } else {
      H.cbeg.assign(size_t(nb), 0);
      H.cend.assign(size_t(nb), 0);
    }
  }
}

std::vector<PairRec> level_pairs_device(const DevTree& DT, int D, int l, DevBuf& fields) {
  std::vector<PairRec> out;
  if (l < 1) return out;
  const int e2 = D - l;  // log2(2w)
  const LvView L = view_of(DT, l), U = view_of(DT, l - 1);
  DevBuf noff;
  const int nnoff = upload_offsets(near_offsets_e2(e2 + 1), noff);
  DevBuf cnt, off;
  cnt.alloc(sizeof(int) * size_t(std::max(1, L.nb)));
  hipLaunchKernelGGL((k_pairs<0>), dim3(nblk(L.nb)), dim3(kBS), 0, 0, L, U, e2, noff.as<int>(), nnoff,
                     cnt.as<int>(), nullptr, nullptr);
  const int64_t np = offsets_of(cnt, off, L.nb);
  fields.alloc(sizeof(int) * 7 * size_t(std::max<int64_t>(1, np)));
  if (np == 0) return out;
  DevBuf k0, k1;
  k0.alloc(sizeof(unsigned long long) * size_t(np));
  k1.alloc(sizeof(unsigned long long) * size_t(np));
  hipLaunchKernelGGL((k_pairs<1>), dim3(nblk(L.nb)), dim3(kBS), 0, 0, L, U, e2, noff.as<int>(), nnoff, nullptr,
                     off.as<int>(), k0.as<unsigned long long>());
  sort_keys_u64(k0.as<unsigned long long>(), k1.as<unsigned long long>(), np, 64);
  hipLaunchKernelGGL(k_pair_fields, dim3(nblk(np)), dim3(kBS), 0, 0, k1.as<unsigned long long>(), np, L, e2,
                     fields.as<int>());
  DFMM_HIP(hipGetLastError());
  std::vector<int> h = download<int>(fields, 7 * np);
  out.resize(size_t(np));
  for (int64_t i = 0; i < np; ++i) {
    const int* r = &h[size_t(7 * i)];
    out[size_t(i)] = PairRec{r[0], r[1], r[2], r[3], r[4], r[5], r[6]};
  }
  return out;
}

void near_lists_device(const DevTree& DT, int D, std::vector<int32_t>& start, std::vector<int32_t>& src) {
  const LvView L = view_of(DT, D);
  DevBuf noff;
  const int nnoff = upload_offsets(near_offsets_e2(0), noff);
  DevBuf cnt, off, out;
  cnt.alloc(sizeof(int) * size_t(std::max(1, L.nb)));
  hipLaunchKernelGGL((k_near<0>), dim3(nblk(L.nb)), dim3(kBS), 0, 0, L, noff.as<int>(), nnoff, cnt.as<int>(),
                     nullptr, nullptr);
  const int64_t tot = offsets_of(cnt, off, L.nb);
  out.alloc(sizeof(int) * size_t(std::max<int64_t>(1, tot)));
  hipLaunchKernelGGL((k_near<1>), dim3(nblk(L.nb)), dim3(kBS), 0, 0, L, noff.as<int>(), nnoff, nullptr,
                     off.as<int>(), out.as<int>());
  DFMM_HIP(hipGetLastError());
  std::vector<int> o = download<int>(off, L.nb);
  src = download<int>(out, tot);
  start.assign(o.begin(), o.end());
  start.push_back(int32_t(tot));
}

void slot_closure_device(const DevTree& DT, int D, int l_top, const std::vector<DevBuf>& fields,
                         const std::vector<int64_t>& npairs, std::vector<SlotIndex>& OS,
                         std::vector<SlotIndex>& IS) {
  OS.assign(size_t(D) + 1, {});
  IS.assign(size_t(D) + 1, {});
  if (l_top < 0) return;
  DevBuf pout, pin;  // the parent level's flags
  int ndir_p = 0;
  for (int l = l_top; l < D; ++l) {
    const int64_t w = int64_t(1) << (D - 1 - l);
    const int ndir = int(6 * w * w);
    const LvView L = view_of(DT, l);
    const int64_t nflag = int64_t(L.nb) * ndir;
    DevBuf fo, fi;
    fo.alloc(sizeof(int) * size_t(nflag));
    fi.alloc(sizeof(int) * size_t(nflag));
    DFMM_HIP(hipMemset(fo.p, 0, sizeof(int) * size_t(nflag)));
    DFMM_HIP(hipMemset(fi.p, 0, sizeof(int) * size_t(nflag)));
    if (npairs[size_t(l)] > 0)
      hipLaunchKernelGGL(k_mark_pairs, dim3(nblk(npairs[size_t(l)])), dim3(kBS), 0, 0, fields[size_t(l)].as<int>(),
                         npairs[size_t(l)], ndir, fo.as<int>(), fi.as<int>());
    if (l > l_top) {
      const LvView U = view_of(DT, l - 1);
      hipLaunchKernelGGL(k_mark_down, dim3(nblk(int64_t(U.nb) * ndir_p)), dim3(kBS), 0, 0, pout.as<int>(),
                         pin.as<int>(), U.nb, ndir_p, 2 * w, U.cbeg, U.cend, ndir, fo.as<int>(), fi.as<int>());
    }
    DFMM_HIP(hipGetLastError());
    for (int side = 0; side < 2; ++side) {
      const DevBuf& fl = side ? fi : fo;
      SlotIndex& S = side ? IS[size_t(l)] : OS[size_t(l)];
      DevBuf ids;
      ids.alloc(sizeof(int) * size_t(nflag));
      scan_excl(fl.as<int>(), ids.as<int>(), nflag);
      std::vector<int> hf = download<int>(fl, nflag), hi = download<int>(ids, nflag);
      S.ndir = ndir;
      S.dense.assign(size_t(nflag), -1);
      S.list.clear();
      for (int64_t t = 0; t < nflag; ++t)
        if (hf[size_t(t)]) {
          S.dense[size_t(t)] = hi[size_t(t)];
          S.list.push_back({t / ndir, int(t % ndir)});
        }
    }
    pout = std::move(fo);
    pin = std::move(fi);
    ndir_p = ndir;
  }
}

}  // namespace dfmm
