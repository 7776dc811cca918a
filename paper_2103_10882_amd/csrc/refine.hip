// Block-structured 2:1 refined grid (Sec. 4.1-4.2) with sub-cycled levels.
//
// Every level stores 16^3-cell blocks in slots, populations blocked
// [slot][z][q][16][16] (post-collision deviations, storage type S), two
// buffers per level.  Level l holds its leaf blocks ("interior") and ghost
// blocks: block positions of level l inside level-(l-1) leaves next to a
// level-l leaf; their cells within two level-l cells of the level-l region
// form the ghost band.  Per coarse step, Step(l):
//   explode level l into the ghost blocks of l+1 (each fine cell copies its
//   parent's 19 populations); Step(l+1) twice; then the level-l sweep:
//   interior cells pull and collide (omega_l from acoustic scaling), ghost
//   cells stream only; cells next to the finer region take the coalescence
//   pull from a precomputed table: the coarse source keeps the fraction
//   (1 - n_in/8) that did not cut into the finer region, and the fine
//   populations that left the finer region into the ghost cells of the cell
//   are added with weight 1/8.
// The particle lives on the finest level; its coupling runs the same kernels
// as on the uniform grid through block addressing (BAddr).  Blocks near the
// particle are held on the finest level; the layout is re-checked every
// check_every coarse steps and data moves between levels by copying a cell to
// its children or averaging them.  Domains are periodic.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

#include "common.hpp"
#include "uniform.hpp"
#include "stencil.hpp"
#include "particle.hpp"
#include "context.hpp"

namespace vm {

namespace {

constexpr uint8_t kIface = 0x10;   // interior cell with a coalescence pull
// deepest hierarchy, that of the paper's deepest setups (9 levels): the
// per-level seeds step by 16 per finest step, and the migration kernel takes
// per-level tables by value.  The layout is dense over finest block
// positions (at most 2^26 of them), which bounds the coarse domain that deep
// hierarchies can take: one coarse block at 9 levels.
constexpr int kMaxLevels = 9;
// words per slot of the neighbour table: the slots of the 27 blocks around
// it (-1 or -2 where the level stores none), whether all 27 are stored, and
// padding to 128 bytes
constexpr int kNbrWords = 32;

struct IfaceEntry {
  int slot, local;      // the coarse cell
  int fine_slot;        // level-(l+1) slot holding its 8 children (-1 if unused)
  int fine_local;       // local index of child (0,0,0)
  uint32_t src[kQ];     // pull source x - c_q as slot * 4096 + local (unused where weight is 0)
  float weight[kQ];     // weight of the plain pull from the coarse source
  uint8_t mask[kQ];     // children whose value is added with weight 1/8
  uint8_t pad[1];
};

struct LevelParams {
  double sp, sm, sb, F[3];
};

}  // namespace

struct Forest {
  int L = 0;
  int nb0[3] = {0, 0, 0};     // coarse block positions
  int nbL[3] = {0, 0, 0};     // finest block positions
  std::vector<int8_t> leaf, base;
  std::vector<int> boxes;     // sphere block ranges the current layout was built for
  bool flow = false;          // curl-sensor criterion on
  int refinements = 0;
  int prebuilt_taken = 0;     // re-refinements whose tables a host thread built ahead
  long long coarse_steps = 0;
  bool side_pending = false;  // a particle update runs on the side stream
  DevParticle* host_parts = nullptr;  // pinned copy of the particle records for the layout check
  struct Lev {
    int n[3] = {0, 0, 0}, nb[3] = {0, 0, 0};
    long npos = 0;
    int cap = 0, iface_cap = 0;
    std::vector<int> slot_of;         // per block position: slot, -1 coarser, -2 finer
    std::vector<int> interior, ghost; // slot lists
    std::vector<int> pos;             // per slot: x, y, z block position
    std::vector<int> nbr;             // per slot, kNbrWords: the 27 neighbour slots, then all stored (1/0)
    std::vector<int> explode;         // per ghost slot: ghost slot, parent slot, ox, oy, oz
    std::vector<uint16_t> band;       // ghost cells (local index) of each ghost block, in ghost order
    std::vector<int> band_off;        // per ghost block: start in band; one extra end entry
    std::vector<uint32_t> band_dirs;  // per band cell: populations written by explosion, sub-step 1, 2
    std::vector<IfaceEntry> iface;
    LevelParams lp{};
    // device
    size_t off_nbr = 0;
    size_t off_pdf[2] = {0, 0}, off_flags = 0, off_slot_of[2] = {0, 0}, off_pos = 0, off_int = 0, off_ghost = 0,
           off_explode = 0, off_iface = 0, off_band = 0, off_band_off = 0, off_band_dirs = 0, off_vel = 0,
           off_sens = 0;
    int cur = 0, tab = 0;
    int n_int = 0, n_ghost = 0, n_iface = 0;
  };
  std::vector<Lev> lv;
  size_t off_owner = 0, off_leaf[2] = {0, 0};
  int leaf_tab = 0;
  // Host tables of a predicted next layout: the sphere block ranges it is
  // for, its leaf field and every level's tables (rc: the build's result).
  // A host thread (job) builds them while the device steps; the layout
  // check takes them when the ranges it finds are these.
  struct Prebuilt {
    std::vector<int> box;
    std::vector<int8_t> leaf;
    std::vector<Lev> lv;
    int rc = 0;
  };
  std::shared_ptr<Prebuilt> pre;
  std::thread job;
  ~Forest() {
    if (job.joinable()) job.join();
  }
  int wrap(int v, int n) const { return ((v % n) + n) % n; }
  long lpos(int i, int j, int k) const { return ((long)k * nbL[1] + j) * nbL[0] + i; }
  // leaf level of the region holding level-l block position (bi, bj, bk)
  int leaf_block(const std::vector<int8_t>& lf, int l, int bi, int bj, int bk) const {
    const Lev& V = lv[l];
    bi = wrap(bi, V.nb[0]); bj = wrap(bj, V.nb[1]); bk = wrap(bk, V.nb[2]);
    const int s = L - l;
    return lf[lpos(bi << s, bj << s, bk << s)];
  }
};

namespace {

enum CellKind { K_INTERIOR, K_GHOST, K_COARSER, K_FINER };

// Cell kinds of every level for the current leaf field and slot tables.
// Leaves per block position are cached (octree: all finest positions under a
// block agree on "== l" and "> l").  A cell inside a level-(l-1) leaf is a
// ghost when its parent has a level-l leaf among its 27 neighbours; the parent
// neighbourhood of local cell x spans level-l cells 2(x>>1)-2 .. 2(x>>1)+3,
// i.e. the own block and the block below for x < 2, above for x > 13.  Only
// ghost blocks hold ghost cells; their kinds are tabulated once per layout.
struct Kinds {
  const Forest& f;
  std::vector<std::vector<int8_t>> lb;
  std::vector<std::vector<uint8_t>> gk;   // per level: [ghost slot - n_int][4096]
  explicit Kinds(const Forest& fr) : f(fr), lb(fr.L + 1), gk(fr.L + 1) {
    for (int l = 0; l <= f.L; ++l) {
      const Forest::Lev& V = f.lv[l];
      lb[l].resize((size_t)V.npos);
      for (int k = 0; k < V.nb[2]; ++k)
        for (int j = 0; j < V.nb[1]; ++j)
          for (int i = 0; i < V.nb[0]; ++i)
            lb[l][((size_t)k * V.nb[1] + j) * V.nb[0] + i] = (int8_t)f.leaf_block(f.leaf, l, i, j, k);
    }
  }
  static int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
  size_t bpos(int l, int bi, int bj, int bk) const {
    const Forest::Lev& V = f.lv[l];
    bi = wrap1(bi, V.nb[0]); bj = wrap1(bj, V.nb[1]); bk = wrap1(bk, V.nb[2]);
    return ((size_t)bk * V.nb[1] + bj) * V.nb[0] + bi;
  }
  int block(int l, int bi, int bj, int bk) const { return lb[l][bpos(l, bi, bj, bk)]; }
  // after the slot tables of every level are set
  void tabulate_ghosts() {
    for (int l = 1; l <= f.L; ++l) {
      const Forest::Lev& V = f.lv[l];
      const size_t n_int = V.interior.size();
      gk[l].assign(V.ghost.size() * kBlockCells, K_COARSER);
      for (size_t g = 0; g < V.ghost.size(); ++g) {
        const int s = V.ghost[g];
        const int bi = V.pos[3 * s], bj = V.pos[3 * s + 1], bk = V.pos[3 * s + 2];
        bool nb[27];
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx)
              nb[(dz + 1) * 9 + (dy + 1) * 3 + dx + 1] = block(l, bi + dx, bj + dy, bk + dz) == l;
        uint8_t* out = gk[l].data() + (size_t)(s - n_int) * kBlockCells;
        for (int z = 0; z < kBlock; ++z) {
          const int z0 = z < 2 ? 0 : 1, z1 = z > 13 ? 2 : 1;
          for (int y = 0; y < kBlock; ++y) {
            const int y0 = y < 2 ? 0 : 1, y1 = y > 13 ? 2 : 1;
            for (int x = 0; x < kBlock; ++x) {
              const int x0 = x < 2 ? 0 : 1, x1 = x > 13 ? 2 : 1;
              bool g2 = false;
              for (int c = z0; c <= z1 && !g2; ++c)
                for (int b = y0; b <= y1 && !g2; ++b)
                  for (int a = x0; a <= x1 && !g2; ++a) g2 = nb[c * 9 + b * 3 + a];
              out[(z * kBlock + y) * kBlock + x] = g2 ? K_GHOST : K_COARSER;
            }
          }
        }
      }
    }
  }
  int kind(int l, int i, int j, int k) const {
    const Forest::Lev& V = f.lv[l];
    i = wrap1(i, V.n[0]); j = wrap1(j, V.n[1]); k = wrap1(k, V.n[2]);
    const size_t p = ((size_t)(k >> 4) * V.nb[1] + (j >> 4)) * V.nb[0] + (i >> 4);
    const int lf = lb[l][p];
    if (lf == l) return K_INTERIOR;
    if (lf > l) return K_FINER;
    if (lf < l - 1) return K_COARSER;
    const int s = V.slot_of[p];
    if (s < 0) return K_COARSER;
    return gk[l][(size_t)(s - (int)V.interior.size()) * kBlockCells + (((k & 15) * kBlock + (j & 15)) * kBlock + (i & 15))];
  }
  // any level-l cell in [i-2, i+2]^3 inside a finer leaf
  bool near_finer(int l, int i, int j, int k) const {
    const Forest::Lev& V = f.lv[l];
    int b0[3], b1[3];
    const int c[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) {
      b0[a] = wrap1(c[a] - 2, V.n[a]) >> 4;
      b1[a] = wrap1(c[a] + 2, V.n[a]) >> 4;
    }
    for (int z = 0; z < 2; ++z)
      for (int y = 0; y < 2; ++y)
        for (int x = 0; x < 2; ++x)
          if (block(l, x ? b1[0] : b0[0], y ? b1[1] : b0[1], z ? b1[2] : b0[2]) > l) return true;
    return false;
  }
};

// Leaf level per finest block position from targets: a node of level l is
// split when any target inside exceeds l; leaves touched (face, edge or
// corner) by leaves more than one level finer are split too, until nothing
// changes.
std::vector<int8_t> balance_layout(const Forest& f, std::vector<int8_t> t) {
  const int L = f.L;
  const long NB = (long)f.nbL[0] * f.nbL[1] * f.nbL[2];
  std::vector<int8_t> lf(NB, 0);
  // pyramid of maxima: level-l node (edge 2^(L-l) positions)
  auto node_dims = [&](int l, int d[3]) { for (int a = 0; a < 3; ++a) d[a] = f.nbL[a] >> (L - l); };
  std::vector<std::vector<int8_t>> mx(L + 1);
  // each pass splits violating leaves by one level: at most L passes per
  // level of difference, so L * L passes suffice
  for (int iter = 0; iter <= L * L + 64; ++iter) {
    mx[L] = t;
    for (int l = L - 1; l >= 0; --l) {
      int d[3], e[3];
      node_dims(l, d);
      node_dims(l + 1, e);
      mx[l].assign((long)d[0] * d[1] * d[2], 0);
      for (int k = 0; k < e[2]; ++k)
        for (int j = 0; j < e[1]; ++j)
          for (int i = 0; i < e[0]; ++i) {
            int8_t& m = mx[l][((long)(k >> 1) * d[1] + (j >> 1)) * d[0] + (i >> 1)];
            m = std::max(m, mx[l + 1][((long)k * e[1] + j) * e[0] + i]);
          }
    }
    // leaf of a position: first level whose node holds no target beyond it
    for (int k = 0; k < f.nbL[2]; ++k)
      for (int j = 0; j < f.nbL[1]; ++j)
        for (int i = 0; i < f.nbL[0]; ++i) {
          int l = 0;
          while (l < L) {
            int d[3];
            node_dims(l, d);
            const int s = L - l;
            if (mx[l][((long)(k >> s) * d[1] + (j >> s)) * d[0] + (i >> s)] <= l) break;
            ++l;
          }
          lf[f.lpos(i, j, k)] = (int8_t)l;
        }
    // 2:1: the deepest leaf touching each leaf node (face, edge or corner)
    // lies in the one-position shell around it
    bool changed = false;
    for (int k = 0; k < f.nbL[2]; ++k)
      for (int j = 0; j < f.nbL[1]; ++j)
        for (int i = 0; i < f.nbL[0]; ++i) {
          const int l = lf[f.lpos(i, j, k)];
          const int S = 1 << (L - l);
          if ((i & (S - 1)) || (j & (S - 1)) || (k & (S - 1))) continue;   // node origin only
          int m = 0;
          for (int c = -1; c <= S; ++c)
            for (int b = -1; b <= S; ++b)
              for (int a = -1; a <= S; ++a) {
                if (a >= 0 && a < S && b >= 0 && b < S && c >= 0 && c < S) continue;
                m = std::max(m, (int)lf[f.lpos(f.wrap(i + a, f.nbL[0]), f.wrap(j + b, f.nbL[1]),
                                               f.wrap(k + c, f.nbL[2]))]);
              }
          // split once; the next pass checks the children
          if (m > l + 1)
            for (int c = 0; c < S; ++c)
              for (int b = 0; b < S; ++b)
                for (int a = 0; a < S; ++a) {
                  int8_t& tv = t[f.lpos(i + a, j + b, k + c)];
                  if (tv < l + 1) { tv = (int8_t)(l + 1); changed = true; }
                }
        }
    if (!changed) return lf;
  }
  return lf;
}

// finest block ranges [lo, hi] meeting the open box (x - r - b, x + r + b) of
// every sphere: the layout is a function of these ranges and the static
// regions only
std::vector<int> sphere_boxes(const std::vector<vmlbm_sphere>& sph) {
  const int b = kBlock;
  std::vector<int> box;
  box.reserve(6 * sph.size());
  for (const auto& s : sph) {
    for (int a = 0; a < 3; ++a) box.push_back((int)std::floor((s.x[a] - s.radius - b) / b));
    for (int a = 0; a < 3; ++a) box.push_back((int)std::ceil((s.x[a] + s.radius + b) / b) - 1);
  }
  return box;
}

std::vector<int8_t> layout_targets(const Forest& f, const std::vector<int>& box) {
  std::vector<int8_t> t = f.base;
  for (size_t s = 0; s < box.size(); s += 6) {
    const int* lo = &box[s];
    const int* hi = &box[s + 3];
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i)
          t[f.lpos(f.wrap(i, f.nbL[0]), f.wrap(j, f.nbL[1]), f.wrap(k, f.nbL[2]))] = (int8_t)f.L;
  }
  return t;
}

// Coalescence entries of one interior level-l block next to the finer
// region.  Returns 0, 1 (a cell pulls from an uncovered coarser cell) or 2
// (children of a coalescence cell are not in a ghost block).
int iface_block(const Kinds& K, const Forest& f, int l, int s, std::vector<IfaceEntry>& out) {
  const Forest::Lev& V = f.lv[l];
  const Forest::Lev& Fl = f.lv[l + 1];
  const int bi = V.pos[3 * s], bj = V.pos[3 * s + 1], bk = V.pos[3 * s + 2];
  for (int lz = 0; lz < kBlock; ++lz)
    for (int ly = 0; ly < kBlock; ++ly)
      for (int lx = 0; lx < kBlock; ++lx) {
        const int i = bi * kBlock + lx, j = bj * kBlock + ly, k = bk * kBlock + lz;
        if (!K.near_finer(l, i, j, k)) continue;
        IfaceEntry e{};
        bool special = false, anymask = false;
        int child_kind[8];
        for (int m = 0; m < 8; ++m)
          child_kind[m] = K.kind(l + 1, 2 * i + (m & 1), 2 * j + ((m >> 1) & 1), 2 * k + (m >> 2));
        for (int q = 0; q < kQ; ++q) {
          const int cq[3] = {cx_of(q), cy_of(q), cz_of(q)};
          const int si = i - cq[0], sj = j - cq[1], sk = k - cq[2];
          const int ks = K.kind(l, si, sj, sk);
          float wgt = 1.0f;
          e.src[q] = 0;
          if (ks == K_INTERIOR || ks == K_GHOST) {
            const int wi = Kinds::wrap1(si, V.n[0]), wj = Kinds::wrap1(sj, V.n[1]), wk = Kinds::wrap1(sk, V.n[2]);
            const int ss = V.slot_of[K.bpos(l, wi >> 4, wj >> 4, wk >> 4)];
            if (ss < 0) return 1;
            e.src[q] = (uint32_t)ss * kBlockCells + (uint32_t)(((wk & 15) * 16 + (wj & 15)) * 16 + (wi & 15));
          }
          if (ks == K_INTERIOR) {
            int nin = 0;
            for (int m = 0; m < 8; ++m) {
              const int gi = 2 * si + (m & 1), gj = 2 * sj + ((m >> 1) & 1), gk = 2 * sk + (m >> 2);
              if (K.kind(l + 1, gi + cq[0], gj + cq[1], gk + cq[2]) == K_INTERIOR) ++nin;
            }
            wgt = 1.0f - nin / 8.0f;
          } else if (ks == K_FINER) {
            wgt = 0.0f;
          } else if (ks == K_COARSER) {
            return 1;
          }
          uint8_t mask = 0;
          for (int m = 0; m < 8; ++m) {
            if (child_kind[m] != K_GHOST) continue;
            const int gi = 2 * i + (m & 1), gj = 2 * j + ((m >> 1) & 1), gk = 2 * k + (m >> 2);
            const int k1 = K.kind(l + 1, gi - cq[0], gj - cq[1], gk - cq[2]);
            if (k1 == K_INTERIOR ||
                (k1 == K_GHOST && K.kind(l + 1, gi - 2 * cq[0], gj - 2 * cq[1], gk - 2 * cq[2]) == K_INTERIOR))
              mask |= (uint8_t)(1u << m);
          }
          e.weight[q] = wgt;
          e.mask[q] = mask;
          special = special || wgt != 1.0f || mask;
          anymask = anymask || mask;
        }
        if (!special) continue;
        e.slot = s;
        e.local = (lz * kBlock + ly) * kBlock + lx;
        e.fine_slot = -1;
        e.fine_local = 0;
        if (anymask) {
          const int fi = 2 * i, fj = 2 * j, fk = 2 * k;
          const long fp = ((long)(fk >> 4) * Fl.nb[1] + (fj >> 4)) * Fl.nb[0] + (fi >> 4);
          const int fs = Fl.slot_of[fp];
          if (fs < (int)Fl.interior.size()) return 2;
          e.fine_slot = fs;
          e.fine_local = (((fk & 15) * kBlock) + (fj & 15)) * kBlock + (fi & 15);
        }
        out.push_back(e);
      }
  return 0;
}

// Per-level block-slot and coalescence-table capacities for every position
// the spheres can reach.  The layout around one sphere is unchanged by a
// shift of a whole coarse node (2^L finest blocks), it grows with the width
// of the sphere's block range, and for a box of targets the 2:1 balance acts
// on each axis separately.  Hence the per-axis extent of each level's region
// (leaves of that level or finer), maximised over the 2^L offsets of the
// widest block range within a coarse node, bounds the region for any
// position; slots lie within one block of it, coalescence cells in the
// blocks next to the finer region.  Spheres add their bounds to the blocks
// the static regions need.
void plan_capacity(vmlbm_ctx* c, Forest& f, std::vector<long>& cap, std::vector<long>& icap) {
  const int L = f.L, b = kBlock;
  cap.assign(L + 1, 0);
  icap.assign(L + 1, 0);
  // blocks of the static regions alone
  {
    const std::vector<int8_t> keep = f.leaf;
    f.leaf = balance_layout(f, f.base);
    Kinds K(f);
    for (int l = 0; l <= L; ++l) {
      const Forest::Lev& V = f.lv[l];
      for (int k = 0; k < V.nb[2]; ++k)
        for (int j = 0; j < V.nb[1]; ++j)
          for (int i = 0; i < V.nb[0]; ++i) {
            const int lf = K.block(l, i, j, k);
            bool slot = lf == l, near = false;
            for (int dz = -1; dz <= 1; ++dz)
              for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                  const int m = K.block(l, i + dx, j + dy, k + dz);
                  if (l >= 1 && lf == l - 1 && m == l) slot = true;
                  if (lf == l && m > l) near = true;
                }
            cap[l] += slot;
            icap[l] += near ? kBlockCells : 0;
          }
    }
    f.leaf = keep;
  }
  // Spheres: the layout around one sphere repeats under shifts by a whole
  // coarse node, so the offsets of its widest block range within a node
  // (the same along all axes: the extents are per axis) cover every place.
  // Per offset, with B_l the region of leaves at level >= l (in level-l
  // blocks), e_l its per-axis extents and |.| exact counts:
  //   slots at level l (leaves and ghost blocks) <= prod(e_l + 2) - |B_{l+1}|,
  //   coalescence cells of level l <= prod(16 e'_l + 4) - 4096 |B_{l+1}|,
  // where e'_l are the extents of B_{l+1} in level-l blocks: ghost blocks lie
  // in the one-block shell around B_l, coalescence cells within two cells
  // of B_{l+1}.  The offsets run on host threads.
  const int node = 1 << L;   // coarse node edge in finest blocks
  for (const auto& s : c->spheres) {
    const int w = (int)std::ceil(2.0 * (s.radius + b) / b) + 1;   // widest block range
    std::vector<std::vector<long>> oc(node, std::vector<long>(L + 1, 0)), oi(node, std::vector<long>(L + 1, 0));
    auto one_offset = [&](int o) {
      std::vector<int8_t> t(f.base.size(), 0);
      int lo[3];
      for (int a = 0; a < 3; ++a) lo[a] = (f.nbL[a] / 2 / node) * node + o;
      for (int k = 0; k < w; ++k)
        for (int j = 0; j < w; ++j)
          for (int i = 0; i < w; ++i)
            t[f.lpos(f.wrap(lo[0] + i, f.nbL[0]), f.wrap(lo[1] + j, f.nbL[1]), f.wrap(lo[2] + k, f.nbL[2]))] =
                (int8_t)L;
      const std::vector<int8_t> lf = balance_layout(f, t);
      // finest positions per leaf level
      std::vector<long> at(L + 2, 0);
      for (int8_t v : lf) at[v] += 1;
      // |B_m| in level-l blocks = (finest positions with leaf >= m) / 8^(L-l)
      auto count_ge = [&](int m, int l) {
        long n = 0;
        for (int v = m; v <= L; ++v) n += at[v];
        return n >> (3 * (L - l));
      };
      for (int l = 1; l <= L; ++l) {
        // projections of B_l onto the axes, in level-l and level-(l-1) blocks
        const int sh = L - l;
        std::vector<std::vector<char>> pl(3), pc(3);
        for (int a = 0; a < 3; ++a) {
          pl[a].assign(f.lv[l].nb[a], 0);
          pc[a].assign(f.lv[l - 1].nb[a], 0);
        }
        for (int k = 0; k < f.nbL[2]; ++k)
          for (int j = 0; j < f.nbL[1]; ++j)
            for (int i = 0; i < f.nbL[0]; ++i)
              if (lf[f.lpos(i, j, k)] >= l) {
                const int q[3] = {i, j, k};
                for (int a = 0; a < 3; ++a) {
                  pl[a][q[a] >> sh] = 1;
                  pc[a][q[a] >> (sh + 1)] = 1;
                }
              }
        long box = 1, cbox = 1;
        for (int a = 0; a < 3; ++a) {
          const long e = std::count(pl[a].begin(), pl[a].end(), 1);
          const long ep = std::count(pc[a].begin(), pc[a].end(), 1);
          box *= std::min<long>(f.lv[l].nb[a], e + 2);
          cbox *= std::min<long>(f.lv[l - 1].n[a], 16 * ep + 4);
        }
        oc[o][l] = box - (l < L ? count_ge(l + 1, l) : 0);
        oi[o][l - 1] = cbox - 4096 * count_ge(l, l - 1);
      }
    };
    const int nt = (int)std::max(1u, std::min<unsigned>(16, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (int t0 = 0; t0 < nt; ++t0)
      pool.emplace_back([&, t0]() {
        for (int o = t0; o < node; o += nt) one_offset(o);
      });
    for (auto& th : pool) th.join();
    for (int l = 0; l <= L; ++l) {
      long mc = 0, mi = 0;
      for (int o = 0; o < node; ++o) { mc = std::max(mc, oc[o][l]); mi = std::max(mi, oi[o][l]); }
      cap[l] += mc;
      icap[l] += mi;
    }
  }
  for (int l = 0; l <= L; ++l) {
    cap[l] = std::min<long>(f.lv[l].npos, cap[l] + 64);
    icap[l] = std::min<long>((long)cap[l] * kBlockCells, icap[l] + 4096);
    if (f.flow) {
      // the flow decides the layout: every block position, or the caller's cap.
      // Coalescence cells lie within two cells of a leaf block's surface:
      // at most 16^3 - 12^3 per block.
      const int mb = c->cfg.max_blocks;
      cap[l] = mb > 0 ? std::min<long>(f.lv[l].npos, mb) : f.lv[l].npos;
      icap[l] = (long)cap[l] * (kBlockCells - 12 * 12 * 12);
    }
  }
}

// Populations of the ghost band of level l (l >= 1) that are read before the
// next explosion overwrites them; only those are written.  Within one
// level-(l-1) step, with buffers A (current) and B:
//   explosion -> A;  sub-step 1 reads A, writes B;  sub-step 2 reads B,
//   writes A;  the level-(l-1) coalescence reads A.
// Sub-step 2 produces the children its coalescence table adds (bit q of the
// entry's mask).  Sub-step 1 produces population q of band cell g where
// g + c_q is an interior cell (its pull in sub-step 2; coalescence cells of
// level l and the link and second-node reads of the particle coupling are
// such pulls) and the band sources g - c_q of the sub-step-2 streaming.  The
// explosion produces the same for sub-step 1: the interior pulls and the band
// sources of the sub-step-1 streaming.  band_dirs[3 i + s], bit q: band cell i
// writes population q in the explosion (s = 0) or in sub-step s.
void band_directions(const Kinds& K, Forest& f, int l) {
  Forest::Lev& V = f.lv[l];
  const int n_int = (int)V.interior.size();
  const int ng = (int)V.ghost.size();
  V.band_dirs.assign(3 * V.band.size(), 0u);
  std::vector<int> at((size_t)ng * kBlockCells, -1);   // band index of every ghost-block cell
  for (int g = 0; g < ng; ++g)
    for (int i = V.band_off[g]; i < V.band_off[g + 1]; ++i) at[(size_t)g * kBlockCells + V.band[i]] = i;
  // Every band cell writes only its own masks, so ghost blocks are split
  // over host threads.  A cell's neighbours lie in the 27 blocks around its
  // own; whether a cell is interior is a property of its block (leaf level
  // l), so per block only the neighbours' slots and leaf levels are looked up.
  auto over_cells = [&](auto&& fn) {
    const int nt = std::max(1, std::min({ng, 16, (int)std::max(1u, std::thread::hardware_concurrency())}));
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t)
      pool.emplace_back([&, t]() {
        int nslot[27];
        bool ninterior[27];
        for (int g = t; g < ng; g += nt) {
          const int s = V.ghost[g];
          const int bi = V.pos[3 * s], bj = V.pos[3 * s + 1], bk = V.pos[3 * s + 2];
          for (int d = 0; d < 27; ++d) {
            const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
            nslot[d] = V.slot_of[K.bpos(l, bi + dx, bj + dy, bk + dz)];
            ninterior[d] = K.block(l, bi + dx, bj + dy, bk + dz) == l;
          }
          for (int b = V.band_off[g]; b < V.band_off[g + 1]; ++b) {
            const int loc = V.band[b];
            fn(b, loc & 15, (loc >> 4) & 15, loc >> 8, nslot, ninterior);
          }
        }
      });
    for (auto& th : pool) th.join();
  };
  // neighbour block (0..26) and local index of local cell (x, y, z) + c_q
  auto step = [](int x, int y, int z, int q, int& d, int& loc) {
    const int xs = x + cx_of(q), ys = y + cy_of(q), zs = z + cz_of(q);
    const int bx = xs < 0 ? 0 : (xs > 15 ? 2 : 1), by = ys < 0 ? 0 : (ys > 15 ? 2 : 1), bz = zs < 0 ? 0 : (zs > 15 ? 2 : 1);
    d = bz * 9 + by * 3 + bx;
    loc = ((zs & 15) * kBlock + (ys & 15)) * kBlock + (xs & 15);
  };
  // sub-step 2: the coalescence reads of level l - 1
  for (const IfaceEntry& e : f.lv[l - 1].iface) {
    if (e.fine_slot < n_int) continue;
    for (int q = 0; q < kQ; ++q)
      for (int m = 0; m < 8; ++m)
        if (e.mask[q] & (1u << m)) {
          const int loc = e.fine_local + ((m >> 2) * kBlock + ((m >> 1) & 1)) * kBlock + (m & 1);
          const int b = at[(size_t)(e.fine_slot - n_int) * kBlockCells + loc];
          if (b >= 0) V.band_dirs[3 * b + 2] |= 1u << q;
        }
  }
  // sub-step 1 and explosion: the interior pulls, then the band sources of
  // the streaming of the following stage (population q of cell b is such a
  // source when the band cell b + c_q streams q in that stage)
  over_cells([&](int b, int x, int y, int z, const int*, const bool* ninterior) {
    uint32_t pulled = 0;
    for (int q = 1; q < kQ; ++q) {
      int d, loc;
      step(x, y, z, q, d, loc);
      if (ninterior[d]) pulled |= 1u << q;
    }
    V.band_dirs[3 * b] = pulled;
    V.band_dirs[3 * b + 1] = pulled;
  });
  for (int st = 2; st >= 1; --st)
    over_cells([&](int b, int x, int y, int z, const int* nslot, const bool*) {
      uint32_t m = 0;
      for (int q = 1; q < kQ; ++q) {
        int d, loc;
        step(x, y, z, q, d, loc);
        const int s = nslot[d];
        if (s < n_int) continue;
        const int g = at[(size_t)(s - n_int) * kBlockCells + loc];
        if (g >= 0 && (V.band_dirs[3 * g + st] & (1u << q))) m |= 1u << q;
      }
      V.band_dirs[3 * b + st - 1] |= m;
    });
}

// slot lists, ghost blocks, explosion map and coalescence table of every
// level for the current leaf field
int build_tables(vmlbm_ctx* c, Forest& f) {
  const int L = f.L;
  Kinds K(f);
  for (int l = 0; l <= L; ++l) {
    Forest::Lev& V = f.lv[l];
    V.slot_of.assign(V.npos, -1);
    V.interior.clear();
    V.ghost.clear();
    V.pos.clear();
    std::vector<int> gpos;
    for (int k = 0; k < V.nb[2]; ++k)
      for (int j = 0; j < V.nb[1]; ++j)
        for (int i = 0; i < V.nb[0]; ++i) {
          const long p = ((long)k * V.nb[1] + j) * V.nb[0] + i;
          const int lf = K.block(l, i, j, k);
          if (lf == l) {
            V.slot_of[p] = (int)V.interior.size();
            V.interior.push_back(V.slot_of[p]);
            V.pos.insert(V.pos.end(), {i, j, k});
          } else if (lf > l) {
            V.slot_of[p] = -2;
          } else if (l >= 1 && lf == l - 1) {
            bool g = false;
            for (int dz = -1; dz <= 1 && !g; ++dz)
              for (int dy = -1; dy <= 1 && !g; ++dy)
                for (int dx = -1; dx <= 1 && !g; ++dx)
                  if (K.block(l, i + dx, j + dy, k + dz) == l) g = true;
            if (g) gpos.insert(gpos.end(), {i, j, k});
          }
        }
    for (size_t g = 0; g < gpos.size(); g += 3) {
      const int s = (int)(V.pos.size() / 3);
      V.slot_of[((long)gpos[g + 2] * V.nb[1] + gpos[g + 1]) * V.nb[0] + gpos[g]] = s;
      V.ghost.push_back(s);
      V.pos.insert(V.pos.end(), {gpos[g], gpos[g + 1], gpos[g + 2]});
    }
    const int nslots = (int)(V.pos.size() / 3);
    if (V.cap && nslots > V.cap)
      return fail(c, VMLBM_ERANGE, "level %d needs %d block slots, capacity %d", l, nslots, V.cap);
  }
  // neighbour table: per slot, the slots of the 27 blocks around it
  // (periodic), as the level kernels look them up
  for (int l = 0; l <= L; ++l) {
    Forest::Lev& V = f.lv[l];
    const int nslots = (int)(V.pos.size() / 3);
    V.nbr.assign((size_t)nslots * kNbrWords, 0);
    for (int s = 0; s < nslots; ++s) {
      int* e = V.nbr.data() + (size_t)s * kNbrWords;
      int all = 1;
      for (int t = 0; t < 27; ++t) {
        const int bx = Kinds::wrap1(V.pos[3 * s] + t % 3 - 1, V.nb[0]);
        const int by = Kinds::wrap1(V.pos[3 * s + 1] + (t / 3) % 3 - 1, V.nb[1]);
        const int bz = Kinds::wrap1(V.pos[3 * s + 2] + t / 9 - 1, V.nb[2]);
        e[t] = V.slot_of[((long)bz * V.nb[1] + by) * V.nb[0] + bx];
        all &= e[t] >= 0;
      }
      e[27] = all;
    }
  }
  K.tabulate_ghosts();
  // ghost cells of each ghost block
  for (int l = 0; l <= L; ++l) {
    Forest::Lev& V = f.lv[l];
    V.band.clear();
    V.band_off.assign(1, 0);
    if (l == 0) continue;
    for (size_t g = 0; g < V.ghost.size(); ++g) {
      const uint8_t* kd = K.gk[l].data() + g * kBlockCells;
      for (int c = 0; c < kBlockCells; ++c)
        if (kd[c] == K_GHOST) V.band.push_back((uint16_t)c);
      V.band_off.push_back((int)V.band.size());
    }
  }
  // explosion: ghost block of level l+1 -> parent interior block of level l
  for (int l = 1; l <= L; ++l) {
    Forest::Lev& V = f.lv[l];
    const Forest::Lev& P = f.lv[l - 1];
    V.explode.clear();
    for (int g : V.ghost) {
      const int bi = V.pos[3 * g], bj = V.pos[3 * g + 1], bk = V.pos[3 * g + 2];
      const long pp = ((long)(bk >> 1) * P.nb[1] + (bj >> 1)) * P.nb[0] + (bi >> 1);
      const int ps = P.slot_of[pp];
      if (ps < 0 || ps >= (int)P.interior.size())
        return fail(c, VMLBM_ERANGE, "ghost block of level %d without an interior parent", l);
      V.explode.insert(V.explode.end(), {g, ps, (bi & 1) * 8, (bj & 1) * 8, (bk & 1) * 8});
    }
  }
  // coalescence table: interior cells of level l within two cells of the
  // level-(l+1) region whose pull differs from plain streaming; blocks are
  // independent and split over host threads, entries kept in block order
  for (int l = 0; l < L; ++l) {
    Forest::Lev& V = f.lv[l];
    std::vector<int> near;
    for (int s : V.interior) {
      const int bi = V.pos[3 * s], bj = V.pos[3 * s + 1], bk = V.pos[3 * s + 2];
      bool any = false;
      for (int dz = -1; dz <= 1 && !any; ++dz)
        for (int dy = -1; dy <= 1 && !any; ++dy)
          for (int dx = -1; dx <= 1 && !any; ++dx)
            if (K.block(l, bi + dx, bj + dy, bk + dz) > l) any = true;
      if (any) near.push_back(s);
    }
    std::vector<std::vector<IfaceEntry>> part(near.size());
    std::vector<int> err(near.size(), 0);
    const int nt = (int)std::max<size_t>(1, std::min<size_t>({near.size(), 16, (size_t)std::max(1u, std::thread::hardware_concurrency())}));
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t)
      pool.emplace_back([&, t]() {
        for (size_t n = t; n < near.size(); n += nt) err[n] = iface_block(K, f, l, near[n], part[n]);
      });
    for (auto& th : pool) th.join();
    V.iface.clear();
    for (size_t n = 0; n < near.size(); ++n) {
      if (err[n] == 1) return fail(c, VMLBM_ERANGE, "level %d cell pulls from an uncovered coarser cell", l);
      if (err[n] == 2) return fail(c, VMLBM_ERANGE, "coalescence children of level %d not in a ghost block", l);
      V.iface.insert(V.iface.end(), part[n].begin(), part[n].end());
    }
    if (V.iface_cap && (int)V.iface.size() > V.iface_cap)
      return fail(c, VMLBM_ERANGE, "level %d coalescence table needs %zu entries, capacity %d", l, V.iface.size(),
                  V.iface_cap);
  }
  for (int l = 1; l <= L; ++l) band_directions(K, f, l);
  return VMLBM_OK;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
struct LevelArgs {
  int n[3], nb[3];
  const int* slot_of;
  const int* pos;      // per slot: block position x, y, z
  const int* nbr;      // per slot: neighbour table (kNbrWords)
  uint32_t N;          // population stride (cap * 4096)
  double sp, sm, sb, F[3];
  uint32_t seed;       // stochastic-rounding stream of this sweep
};

// population q of local cell (x,y,z) pulled from x - c_q, via the neighbour
// slot table nb[27]; returns false if the source block is not stored
template <typename S, int Q, bool CHECK = true>
__device__ __forceinline__ bool pull_block(const S* __restrict__ src, const int* nbs, int slot, int x, int y, int z,
                                           typename Store<S>::T& out) {
  constexpr int cx = cx_of(Q), cy = cy_of(Q), cz = cz_of(Q);
  int xs = x - cx, ys = y - cy, zs = z - cz;
  const int bx = xs < 0 ? -1 : (xs > 15 ? 1 : 0), by = ys < 0 ? -1 : (ys > 15 ? 1 : 0),
            bz = zs < 0 ? -1 : (zs > 15 ? 1 : 0);
  const int s = (bx | by | bz) ? nbs[(bz + 1) * 9 + (by + 1) * 3 + (bx + 1)] : slot;
  if (CHECK && s < 0) return false;
  const uint32_t c = (uint32_t)s * kBlockCells + (uint32_t)(((zs & 15) * 16 + (ys & 15)) * 16 + (xs & 15));
  out = Store<S>::load(src[bpop(Q, c)]);
  return true;
}

template <typename S, bool CHECK, int... Qs>
__device__ __forceinline__ bool pull_cell(const S* __restrict__ src, const int* nbs, int slot, int x, int y, int z,
                                          typename Store<S>::T (&d)[kQ], std::integer_sequence<int, Qs...>) {
  return (pull_block<S, Qs, CHECK>(src, nbs, slot, x, y, z, d[Qs]) & ...);
}

// the populations of mask `dirs` of a ghost cell; a source block that is not
// stored gives 0.  All loads are issued before the first store.
template <typename S, int Q>
__device__ __forceinline__ void ghost_pull_one(const S* __restrict__ src, const int* nbs, int slot, int x, int y,
                                               int z, uint32_t dirs, typename Store<S>::T& d) {
  if (!((dirs >> Q) & 1u) || !pull_block<S, Q>(src, nbs, slot, x, y, z, d)) d = typename Store<S>::T(0);
}

template <typename S, int... Qs>
__device__ __forceinline__ void ghost_pull(const S* __restrict__ src, const int* nbs, int slot, int x, int y, int z,
                                           uint32_t dirs, typename Store<S>::T (&d)[kQ],
                                           std::integer_sequence<int, Qs...>) {
  (ghost_pull_one<S, Qs>(src, nbs, slot, x, y, z, dirs, d[Qs]), ...);
}

// the 27 neighbour slots of a block and the all-stored word into LDS
// (nbs[28]), one load per lane from the table the host built with the layout
__device__ __forceinline__ void load_neighbours(const LevelArgs& a, int slot, int* nbs) {
  if (threadIdx.x < 28) nbs[threadIdx.x] = a.nbr[(size_t)slot * kNbrWords + threadIdx.x];
  __syncthreads();
}

// Workgroups are dealt to the 8 XCDs round-robin in launch order.  This
// renumbering gives each XCD a contiguous run of work items instead, so that
// blocks next to each other in the (x-fastest) block list share one L2: the
// x-faces of a block pull single cells out of rows of its x-neighbours.  It
// is a bijection of [0, G) for any G.
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t lin, uint32_t G) {
  const uint32_t q8 = G / 8, r8 = G % 8, xcd = lin % 8, ord = lin / 8;
  return xcd * q8 + min(xcd, r8) + ord;
}

// plane z of one block; CHECK: test that the blocks a cell's pulls reach are
// stored (needed only when a neighbour slot is missing)
template <typename S, bool CHECK, bool MRT>
__device__ __forceinline__ void sweep_plane(const S* __restrict__ src, S* __restrict__ dst,
                                            const uint8_t* __restrict__ flags, int* __restrict__ status,
                                            const LevelArgs& a, const int* nbs, int slot, int z) {
  using T = typename Store<S>::T;
  const int x = threadIdx.x & 15, y = (threadIdx.x >> 4) & 15;
  // CHECK: the pulls of a cell reach the face and edge neighbour blocks on
  // its sides (D3Q19 has no body diagonals, so never the corner block); the
  // cell is tested once against those instead of per direction
  const int sx = x == 0 ? -1 : (x == 15 ? 1 : 0), sy = y == 0 ? -1 : (y == 15 ? 1 : 0);
  auto stored = [&](int dx, int dy, int dz) { return nbs[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] >= 0; };
  const bool xy_ok = !CHECK || (stored(sx, 0, 0) && stored(0, sy, 0) && stored(sx, sy, 0));
  {
    const uint32_t c = (uint32_t)slot * kBlockCells + (uint32_t)((z * 16 + y) * 16 + x);
    if (flags[c]) return;
    T d[kQ];
    if constexpr (CHECK && sizeof(S) == 8) {
      // FP64 keeps the per-direction test: the per-cell one costs it
      // registers (occupancy 3 -> 2)
      if (!pull_cell<S, true>(src, nbs, slot, x, y, z, d, std::make_integer_sequence<int, kQ>{})) {
        status[kStatusRange] = 6;
        return;
      }
    } else {
      if (CHECK) {
        const int sz = z == 0 ? -1 : (z == 15 ? 1 : 0);
        if (!(xy_ok && stored(0, 0, sz) && stored(sx, 0, sz) && stored(0, sy, sz))) {
          status[kStatusRange] = 6;
          return;
        }
      }
      pull_cell<S, false>(src, nbs, slot, x, y, z, d, std::make_integer_sequence<int, kQ>{});
    }
    const T drho = lbm_collide<T, MRT>(d, T(a.sp), T(a.sm), T(a.sb), T(a.F[0]), T(a.F[1]), T(a.F[2]));
    if (!(drho == drho)) status[kStatusUnstable] = 1;
    SrBits rb(c, a.seed);
#pragma unroll
    for (int q = 0; q < kQ; ++q) store_nt(&dst[bpop(q, c)], Store<S>::store_sr(d[q], rb.next()));
  }
}

// interior blocks of a level: pull + collide, cells with flags left out.
// One workgroup per plane of a block, one thread per cell: straight-line
// code needs about 60 registers in FP16 and FP32 (124 in FP64) against 109
// (166) for a loop over planes, and holds twice the waves.  FP32 and FP16
// storage number the work XCD-contiguously (3-4 % faster on the 3-level
// workload); FP64 keeps launch order (3 % slower otherwise).  lin: this
// workgroup's index among the n sweep workgroups (16 per block).
template <typename S, bool MRT>
__device__ __forceinline__ void sweep_role(const S* __restrict__ src, S* __restrict__ dst,
                                           const uint8_t* __restrict__ flags, const int* __restrict__ list,
                                           int* __restrict__ status, const LevelArgs& a, uint32_t lin, uint32_t n) {
  __shared__ int nbs[28];
  const uint32_t item = sizeof(S) < 8 ? xcd_contiguous(lin, n) : lin;
  const int slot = list[item >> 4];
  load_neighbours(a, slot, nbs);
  const int z = (int)(item & 15u);
  // one test per workgroup instead of one per direction and cell
  if (nbs[27]) sweep_plane<S, false, MRT>(src, dst, flags, status, a, nbs, slot, z);
  else sweep_plane<S, true, MRT>(src, dst, flags, status, a, nbs, slot, z);
}

// ghost cells (the band of each ghost block listed in band[band_off[g] ..
// band_off[g+1]) as local cell indices): stream only; sources not stored at
// this level give 0.  Cells of a ghost block outside its band are never
// read by an update of this level's region within the two substeps, and a
// band cell writes only the populations of its direction mask for this
// sub-step (dirs, stride 3), the ones read before the next explosion.  Cells
// on the x-faces of the region form 2-cell runs that touch a cache line per
// population, so the masks cut the lines moved by about four.  A band holds a
// few hundred cells: kBandSplit workgroups share one (part: which of them),
// so that each thread takes about one cell.
constexpr int kBandSplit = 2;
template <typename S>
__device__ __forceinline__ void ghost_role(const S* __restrict__ src, S* __restrict__ dst,
                                           const int* __restrict__ list, const int* __restrict__ band_off,
                                           const uint16_t* __restrict__ band, const uint32_t* __restrict__ dirs,
                                           const LevelArgs& a, int g, int part) {
  using T = typename Store<S>::T;
  __shared__ int nbs[28];
  const int slot = list[g];
  load_neighbours(a, slot, nbs);
  const int b1 = band_off[g + 1];
  for (int i = band_off[g] + part * 256 + (int)threadIdx.x; i < b1; i += kBandSplit * 256) {
    const uint32_t m = dirs[3 * i];
    if (!m) continue;
    const int local = band[i];
    const int x = local & 15, y = (local >> 4) & 15, z = local >> 8;
    const uint32_t c = (uint32_t)slot * kBlockCells + (uint32_t)local;
    T d[kQ];
    ghost_pull<S>(src, nbs, slot, x, y, z, m, d, std::make_integer_sequence<int, kQ>{});
#pragma unroll
    for (int q = 1; q < kQ; ++q)
      if ((m >> q) & 1u) dst[bpop(q, c)] = Store<S>::store(d[q]);
  }
}

// explosion: every ghost cell of level l+1 takes its parent's populations
// (level l, current state), those of its explosion mask (dirs, stride 3);
// ghost block g is explode entry g.  The explosions that follow each other
// with no sweep between them (those of levels l, l+1, ... at the start of a
// level-l step) run as one launch: explosion l writes level l+1's ghost
// blocks and explosion l+1 reads its leaf blocks, so they touch disjoint
// slots.  Set k covers workgroups first .. the next set's first - 1.
struct ExplodeSet {
  const void* coarse;
  void* fine;
  const int* ex;
  const int* band_off;
  const uint16_t* band;
  const uint32_t* dirs;
  int first;
};
struct ExplodeChain {
  ExplodeSet set[kMaxLevels - 1];
  int n;
};

template <typename S>
__global__ __launch_bounds__(256) void k_explode(ExplodeChain ch) {
  int k = 0;
  while (k + 1 < ch.n && (int)blockIdx.x >= ch.set[k + 1].first) ++k;
  const ExplodeSet& e = ch.set[k];
  const S* __restrict__ coarse = (const S*)e.coarse;
  S* __restrict__ fine = (S*)e.fine;
  const int g = (int)blockIdx.x - e.first;
  const int* en = e.ex + 5 * g;
  const int gs = en[0], ps = en[1], ox = en[2], oy = en[3], oz = en[4];
  const int b1 = e.band_off[g + 1];
  for (int i = e.band_off[g] + blockIdx.y * blockDim.x + threadIdx.x; i < b1; i += gridDim.y * blockDim.x) {
    const uint32_t m = e.dirs[3 * i];
    if (!m) continue;
    const int local = e.band[i];
    const int x = local & 15, y = (local >> 4) & 15, z = local >> 8;
    const uint32_t cf = (uint32_t)gs * kBlockCells + (uint32_t)local;
    const uint32_t cc = (uint32_t)ps * kBlockCells +
                        (uint32_t)(((oz + (z >> 1)) * 16 + (oy + (y >> 1))) * 16 + (ox + (x >> 1)));
    S v[kQ];
#pragma unroll
    for (int q = 1; q < kQ; ++q)
      if ((m >> q) & 1u) v[q] = coarse[bpop(q, cc)];
#pragma unroll
    for (int q = 1; q < kQ; ++q)
      if ((m >> q) & 1u) fine[bpop(q, cf)] = v[q];
  }
}

// coalescence cells of level l, kIfaceCells per workgroup: first one thread
// per (cell, q) gathers the weighted coarse pull and the 1/8-weighted fine
// ghost children into LDS, then one thread per cell collides and stores.
// 13 cells x 19 populations fill the 256 threads in one pass (16 cells, two
// passes for 48 threads, measured 0.8 % slower on the 3-level workload)
constexpr int kIfaceCells = 13;

template <typename S>
__device__ __forceinline__ void iface_role(const S* __restrict__ src, S* __restrict__ dst,
                                           const S* __restrict__ fine, const IfaceEntry* __restrict__ tab,
                                           int count, int* __restrict__ status, const LevelArgs& a, int wg) {
  using T = typename Store<S>::T;
  __shared__ double pre[kIfaceCells][kQ];
  const int e0 = wg * kIfaceCells;
  const int n = min(kIfaceCells, count - e0);
  // The source and the eight children are loaded in every thread, so that
  // no branch separates the loads: an unused source index is 0 in the
  // table, and a child outside the mask reads element 0 of the fine array.
  for (int p = threadIdx.x; p < n * kQ; p += 256) {
    const int j = p / kQ, q = p - j * kQ;
    const IfaceEntry& e = tab[e0 + j];
    const float wq = e.weight[q];
    const double sv = (double)Store<S>::load(src[bpop(q, e.src[q])]);
    double v = wq != 0.0f ? (double)wq * sv : 0.0;
    const unsigned mk = e.mask[q];
    const uint32_t c0 = (uint32_t)e.fine_slot * kBlockCells + (uint32_t)e.fine_local;
    typename Store<S>::T ch[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const uint32_t cf = (mk & (1u << m)) ? c0 + (uint32_t)(((m >> 2) * 16 + ((m >> 1) & 1)) * 16 + (m & 1)) : 0u;
      ch[m] = Store<S>::load(fine[bpop(q, cf)]);
    }
    if (mk) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < 8; ++m) acc = (mk & (1u << m)) ? acc + (double)ch[m] : acc;
      v += 0.125 * acc;
    }
    pre[j][q] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x >= n) return;
  const IfaceEntry& e = tab[e0 + threadIdx.x];
  T d[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) d[q] = T(pre[threadIdx.x][q]);
  const T drho = lbm_collide<T>(d, T(a.sp), T(a.sm), T(a.sb), T(a.F[0]), T(a.F[1]), T(a.F[2]));
  if (!(drho == drho)) status[kStatusUnstable] = 1;
  const uint32_t c = (uint32_t)e.slot * kBlockCells + (uint32_t)e.local;
  SrBits rb(c, a.seed);
#pragma unroll
  for (int q = 0; q < kQ; ++q) dst[bpop(q, c)] = Store<S>::store_sr(d[q], rb.next());
}

// The work of one level's sweep as one launch: the ghost bands (kBandSplit
// workgroups per ghost block), the coalescence cells (kIfaceCells per
// workgroup), then the interior planes.  The three write disjoint cells of
// the new state and read the current one (the coalescence cells also the
// finer level's), so they need no order among themselves; the short,
// latency-bound ghost and coalescence workgroups go first so that they run
// beside the bulk rather than after it.  The interior part starts at a
// multiple of 8 workgroups (n_lead, the others' count rounded up), so that
// its numbering keeps the launch order's round-robin over the 8 XCDs.
struct LevelRoles {
  uint32_t n_sweep;                 // interior workgroups (16 per block)
  uint32_t n_lead;                  // workgroups before the interior ones
  int n_ghost_wg;                   // ghost workgroups
  int n_iface_wg, n_iface;          // coalescence workgroups and cells
  const void* fine;                 // level l+1 current state
  const IfaceEntry* iface;
  const int* ghost;                 // ghost block slots, then their bands
  const int* band_off;
  const uint16_t* band;
  const uint32_t* dirs;             // direction masks of this sub-step
};

// About 60 vector and 72 scalar registers in FP16 and FP32: 8 waves per
// SIMD (FP64: 114 and 4).  The scalar count matters: with the neighbour
// lookups done in the prologue it was 104, which held FP16 and FP32 at 7.
template <typename S, bool MRT>
__global__ __launch_bounds__(256) void k_level(
    const S* __restrict__ src, S* __restrict__ dst, const uint8_t* __restrict__ flags,
    const int* __restrict__ list, int* __restrict__ status, LevelArgs a, LevelRoles r) {
  uint32_t b = blockIdx.x;
  if (b >= r.n_lead) {
    sweep_role<S, MRT>(src, dst, flags, list, status, a, b - r.n_lead, r.n_sweep);
    return;
  }
  if ((int)b < r.n_ghost_wg) {
    ghost_role<S>(src, dst, r.ghost, r.band_off, r.band, r.dirs, a, (int)(b / kBandSplit), (int)(b % kBandSplit));
    return;
  }
  b -= (uint32_t)r.n_ghost_wg;
  if ((int)b < r.n_iface_wg) iface_role<S>(src, dst, (const S*)r.fine, r.iface, r.n_iface, status, a, (int)b);
}

// The level sweep's access pattern without arithmetic: every cell of the
// level's leaf blocks takes population q from x - c_q through the sweep's
// numbering, neighbour table and block addressing, and stores it, raw, with
// the sweep's streaming stores; no flags, collision or rounding.  A source in
// a block that is not stored gives 0.  A reference for the bandwidth the
// 16^3-block pattern alone reaches.
template <typename S, int Q, bool CHECK>
__device__ __forceinline__ S pull_raw(const S* __restrict__ src, const int* nbs, int slot, int x, int y, int z) {
  constexpr int cx = cx_of(Q), cy = cy_of(Q), cz = cz_of(Q);
  const int xs = x - cx, ys = y - cy, zs = z - cz;
  const int bx = xs < 0 ? -1 : (xs > 15 ? 1 : 0), by = ys < 0 ? -1 : (ys > 15 ? 1 : 0),
            bz = zs < 0 ? -1 : (zs > 15 ? 1 : 0);
  int s = (bx | by | bz) ? nbs[(bz + 1) * 9 + (by + 1) * 3 + (bx + 1)] : slot;
  const bool missing = CHECK && s < 0;
  s = missing ? slot : s;
  const uint32_t c = (uint32_t)s * kBlockCells + (uint32_t)(((zs & 15) * 16 + (ys & 15)) * 16 + (xs & 15));
  const S v = src[bpop(Q, c)];
  return missing ? Store<S>::store(typename Store<S>::T(0)) : v;
}

template <typename S, bool CHECK, int... Qs>
__device__ __forceinline__ void pull_raw_cell(const S* __restrict__ src, S* __restrict__ dst, const int* nbs,
                                              int slot, int x, int y, int z, uint32_t c,
                                              std::integer_sequence<int, Qs...>) {
  const S v[kQ] = {pull_raw<S, Qs, CHECK>(src, nbs, slot, x, y, z)...};
#pragma unroll
  for (int q = 0; q < kQ; ++q) store_nt(&dst[bpop(q, c)], v[q]);
}

template <typename S>
__global__ __launch_bounds__(256) void k_level_pull(const S* __restrict__ src, S* __restrict__ dst,
                                                    const int* __restrict__ list, LevelArgs a, uint32_t n) {
  __shared__ int nbs[28];
  const uint32_t item = sizeof(S) < 8 ? xcd_contiguous(blockIdx.x, n) : blockIdx.x;
  const int slot = list[item >> 4];
  load_neighbours(a, slot, nbs);
  const int z = (int)(item & 15u), x = threadIdx.x & 15, y = (threadIdx.x >> 4) & 15;
  const uint32_t c = (uint32_t)slot * kBlockCells + (uint32_t)((z * 16 + y) * 16 + x);
  if (nbs[27]) pull_raw_cell<S, false>(src, dst, nbs, slot, x, y, z, c, std::make_integer_sequence<int, kQ>{});
  else pull_raw_cell<S, true>(src, dst, nbs, slot, x, y, z, c, std::make_integer_sequence<int, kQ>{});
}

// stored post-collision velocity of every interior cell of a level:
// u = sum_q c_q d_q - F_l / 2, as vel[a * N + c]
template <typename S>
__global__ __launch_bounds__(256) void k_level_velocity(const S* __restrict__ src, const int* __restrict__ list,
                                                        LevelArgs a, double* __restrict__ vel) {
  const int slot = list[blockIdx.x];
  for (int t = threadIdx.x; t < kBlockCells; t += blockDim.x) {
    const uint32_t c = (uint32_t)slot * kBlockCells + (uint32_t)t;
    double j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 1; q < kQ; ++q) {
      const double d = (double)Store<S>::load(src[bpop(q, c)]);
      j[0] += cx_of(q) * d;
      j[1] += cy_of(q) * d;
      j[2] += cz_of(q) * d;
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) vel[(size_t)b * a.N + c] = j[b] - 0.5 * a.F[b];
  }
}

// Curl sensor of Sec. 4.2.2 per interior block: max over its cells of
// |curl u| s^(3/2) (scale = s^(3/2) / (2 s) applied to the central
// differences), evaluated where all six axis neighbours are interior cells
// of the level and, with flags given (finest level), no cell involved is
// solid; 0 if no cell qualifies.
__global__ __launch_bounds__(256) void k_block_curl(const double* __restrict__ vel,
                                                    const uint8_t* __restrict__ flags,
                                                    const int* __restrict__ list, int n_int, LevelArgs a,
                                                    double scale, double* __restrict__ out) {
  __shared__ int nbs[28];
  __shared__ double red[4];
  const int slot = list[blockIdx.x];
  load_neighbours(a, slot, nbs);
  double m = 0.0;
  for (int t = threadIdx.x; t < kBlockCells; t += blockDim.x) {
    const int x = t & 15, y = (t >> 4) & 15, z = t >> 8;
    const uint32_t c = (uint32_t)slot * kBlockCells + (uint32_t)t;
    if (flags && (flags[c] & kSolid)) continue;
    double du[3][3];   // axis, component: u(+) - u(-)
    bool ok = true;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      double up[2][3];
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        int p[3] = {x, y, z};
        p[ax] += sd ? 1 : -1;
        const int bx = p[0] < 0 ? -1 : (p[0] > 15 ? 1 : 0), by = p[1] < 0 ? -1 : (p[1] > 15 ? 1 : 0),
                  bz = p[2] < 0 ? -1 : (p[2] > 15 ? 1 : 0);
        const int s = (bx | by | bz) ? nbs[(bz + 1) * 9 + (by + 1) * 3 + (bx + 1)] : slot;
        uint32_t cn = c;
        if (s < 0 || s >= n_int) ok = false;
        else cn = (uint32_t)s * kBlockCells + (uint32_t)((((p[2] & 15) * 16) + (p[1] & 15)) * 16 + (p[0] & 15));
        if (flags && (flags[cn] & kSolid)) ok = false;
#pragma unroll
        for (int b = 0; b < 3; ++b) up[sd][b] = vel[(size_t)b * a.N + cn];
      }
#pragma unroll
      for (int b = 0; b < 3; ++b) du[ax][b] = up[1][b] - up[0][b];
    }
    if (!ok) continue;
    const double cx = du[1][2] - du[2][1], cy = du[2][0] - du[0][2], cz = du[0][1] - du[1][0];
    m = fmax(m, sqrt(cx * cx + cy * cy + cz * cz) * scale);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) out[slot] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ void k_mark_iface(uint8_t* __restrict__ flags, const IfaceEntry* __restrict__ tab, int count) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  flags[(uint32_t)tab[t].slot * kBlockCells + (uint32_t)tab[t].local] |= kIface;
}

// f~(0) = collide(f^eq(rho, u)) on every cell of every slot of a level, u of
// the coarse cell holding it
template <typename S>
__global__ __launch_bounds__(256) void k_init_level(S* __restrict__ dst, const double* __restrict__ u0, int l,
                                                    int n0x, int n0y, uint32_t N0, double drho, LevelArgs a) {
  using T = typename Store<S>::T;
  const int slot = blockIdx.x;
  const int* p3 = a.pos + 3 * slot;
  const int x = threadIdx.x & 15, y = threadIdx.x >> 4;
  for (int z = 0; z < kBlock; ++z) {
    const int i = p3[0] * 16 + x, j = p3[1] * 16 + y, k = p3[2] * 16 + z;
    double u[3] = {0.0, 0.0, 0.0};
    if (u0) {
      const uint32_t c0 = ((uint32_t)(k >> l) * n0y + (j >> l)) * n0x + (i >> l);
      u[0] = u0[c0]; u[1] = u0[N0 + c0]; u[2] = u0[2 * (size_t)N0 + c0];
    }
    const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    T d[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const double cu = cx_of(q) * u[0] + cy_of(q) * u[1] + cz_of(q) * u[2];
      d[q] = T(w_of(q) * (drho + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq));
    }
    lbm_collide<T>(d, T(a.sp), T(a.sm), T(a.sb), T(a.F[0]), T(a.F[1]), T(a.F[2]));
    const uint32_t c = (uint32_t)slot * kBlockCells + (uint32_t)((z * 16 + y) * 16 + x);
    SrBits rb(c, a.seed);
#pragma unroll
    for (int q = 0; q < kQ; ++q) dst[bpop(q, c)] = Store<S>::store_sr(d[q], rb.next());
  }
}

// mapping of the finest level's interior slots
__global__ __launch_bounds__(256) void k_map_level(uint8_t* __restrict__ flags, uint16_t* __restrict__ owner,
                                                   const DevParticle* __restrict__ parts, int np, SweepParams p,
                                                   BAddr ad, const int* __restrict__ pos, int* __restrict__ status) {
  const int slot = blockIdx.x;
  const int x = threadIdx.x & 15, y = threadIdx.x >> 4;
  for (int z = 0; z < kBlock; ++z) {
    const int i = pos[3 * slot] * 16 + x, j = pos[3 * slot + 1] * 16 + y, k = pos[3 * slot + 2] * 16 + z;
    const uint32_t c = (uint32_t)slot * kBlockCells + (uint32_t)((z * 16 + y) * 16 + x);
    map_cell<BAddr>(i, j, k, c, flags, owner, parts, np, p, ad, status);
  }
}

// Data of one new interior slot of level l from the old layout: the old leaf
// holding each cell gives the source level; coarser sources are copied,
// finer ones averaged.
struct MigrateArgs {
  int L;
  int nbL[3];
  const int8_t* old_leaf;
  const void* old_pdf[kMaxLevels];
  const int* old_slot_of[kMaxLevels];
  int nb[kMaxLevels][3];
  uint32_t seed;
};

template <typename S>
__global__ __launch_bounds__(256) void k_migrate(S* __restrict__ dst, const int* __restrict__ list,
                                                 const int* __restrict__ pos, int l, MigrateArgs m,
                                                 int* __restrict__ status) {
  const int slot = list[blockIdx.x];
  const int x = threadIdx.x & 15, y = threadIdx.x >> 4;
  for (int z = 0; z < kBlock; ++z) {
    const int i = pos[3 * slot] * 16 + x, j = pos[3 * slot + 1] * 16 + y, k = pos[3 * slot + 2] * 16 + z;
    const int s = m.L - l;
    const int fi = (i << s) >> 4, fj = (j << s) >> 4, fk = (k << s) >> 4;   // finest block position
    const int lo = m.old_leaf[((long)fk * m.nbL[1] + fj) * m.nbL[0] + fi];
    const uint32_t c = (uint32_t)slot * kBlockCells + (uint32_t)((z * 16 + y) * 16 + x);
    double v[kQ];
    for (int q = 0; q < kQ; ++q) v[q] = 0.0;
    bool ok = true;
    if (lo <= l) {
      const int sh = l - lo;
      const int ci = i >> sh, cj = j >> sh, ck = k >> sh;
      const int os = m.old_slot_of[lo][((long)(ck >> 4) * m.nb[lo][1] + (cj >> 4)) * m.nb[lo][0] + (ci >> 4)];
      if (os < 0) ok = false;
      else {
        const uint32_t oc = (uint32_t)os * kBlockCells + (uint32_t)(((ck & 15) * 16 + (cj & 15)) * 16 + (ci & 15));
        const S* src = (const S*)m.old_pdf[lo];
        for (int q = 0; q < kQ; ++q) v[q] = (double)Store<S>::load(src[bpop(q, oc)]);
      }
    } else {
      const int sh = lo - l, e = 1 << sh;
      const S* src = (const S*)m.old_pdf[lo];
      for (int dz = 0; dz < e && ok; ++dz)
        for (int dy = 0; dy < e && ok; ++dy)
          for (int dx = 0; dx < e && ok; ++dx) {
            const int ci = (i << sh) + dx, cj = (j << sh) + dy, ck = (k << sh) + dz;
            const int os = m.old_slot_of[lo][((long)(ck >> 4) * m.nb[lo][1] + (cj >> 4)) * m.nb[lo][0] + (ci >> 4)];
            if (os < 0) { ok = false; break; }
            const uint32_t oc = (uint32_t)os * kBlockCells + (uint32_t)(((ck & 15) * 16 + (cj & 15)) * 16 + (ci & 15));
            for (int q = 0; q < kQ; ++q) v[q] += (double)Store<S>::load(src[bpop(q, oc)]);
          }
      const double inv = 1.0 / (double)(e * e * e);
      for (int q = 0; q < kQ; ++q) v[q] *= inv;
    }
    if (!ok) status[kStatusRange] = 8;
    SrBits rb(c, m.seed);
    for (int q = 0; q < kQ; ++q) dst[bpop(q, c)] = Store<S>::store_sr((typename Store<S>::T)v[q], rb.next());
  }
}

void forest_free(Forest* f) {
  if (f && f->host_parts) (void)hipHostFree(f->host_parts);
  delete f;
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {

LevelArgs level_args(vmlbm_ctx* c, int l, int tab) {
  Forest& f = *c->forest;
  Forest::Lev& V = f.lv[l];
  LevelArgs a{};
  for (int i = 0; i < 3; ++i) { a.n[i] = V.n[i]; a.nb[i] = V.nb[i]; }
  a.slot_of = (const int*)(c->ws + V.off_slot_of[tab]);
  a.pos = (const int*)(c->ws + V.off_pos);
  a.nbr = (const int*)(c->ws + V.off_nbr);
  a.N = (uint32_t)V.cap * kBlockCells;
  a.sp = V.lp.sp;
  a.sm = V.lp.sm;
  a.sb = V.lp.sb;
  for (int i = 0; i < 3; ++i) a.F[i] = V.lp.F[i];
  a.seed = level_seed(c->fine_steps_done, l);
  return a;
}

BAddr finest_addr(vmlbm_ctx* c) {
  Forest& f = *c->forest;
  Forest::Lev& V = f.lv[f.L];
  BAddr ad{};
  for (int i = 0; i < 3; ++i) { ad.n[i] = V.n[i]; ad.nb[i] = V.nb[i]; }
  ad.slot_of = (const int*)(c->ws + V.off_slot_of[V.tab]);
  ad.N = (uint32_t)V.cap * kBlockCells;
  return ad;
}

SweepParams finest_params(vmlbm_ctx* c) {
  Forest& f = *c->forest;
  Forest::Lev& V = f.lv[f.L];
  SweepParams p{};
  p.nx = V.n[0]; p.ny = V.n[1]; p.nz = V.n[2];
  p.per[0] = p.per[1] = p.per[2] = 1;
  p.wall_axis = -1;
  p.sp = V.lp.sp;
  p.sm = V.lp.sm;
  p.sb = V.lp.sb;
  for (int i = 0; i < 3; ++i) p.F[i] = V.lp.F[i];
  p.N = (uint32_t)V.cap * kBlockCells;
  p.box = c->box;
  p.slot_stride = c->slot_stride;
  p.seed = level_seed(c->fine_steps_done, f.L);
  return p;
}

// upload the tables of the current layout; slot_of goes into each level's
// current table set (the other set may still hold the previous layout)
int upload_tables(vmlbm_ctx* c) {
  Forest& f = *c->forest;
  for (int l = 0; l <= f.L; ++l) {
    Forest::Lev& V = f.lv[l];
    HIP_TRY(c, hipMemcpy(c->ws + V.off_slot_of[V.tab], V.slot_of.data(), V.npos * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->ws + V.off_pos, V.pos.data(), V.pos.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!V.nbr.empty())
      HIP_TRY(c, hipMemcpy(c->ws + V.off_nbr, V.nbr.data(), V.nbr.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!V.interior.empty())
      HIP_TRY(c, hipMemcpy(c->ws + V.off_int, V.interior.data(), V.interior.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!V.ghost.empty())
      HIP_TRY(c, hipMemcpy(c->ws + V.off_ghost, V.ghost.data(), V.ghost.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!V.explode.empty())
      HIP_TRY(c, hipMemcpy(c->ws + V.off_explode, V.explode.data(), V.explode.size() * sizeof(int),
                           hipMemcpyHostToDevice));
    if (!V.iface.empty())
      HIP_TRY(c, hipMemcpy(c->ws + V.off_iface, V.iface.data(), V.iface.size() * sizeof(IfaceEntry),
                           hipMemcpyHostToDevice));
    if (!V.band.empty()) {
      HIP_TRY(c, hipMemcpy(c->ws + V.off_band, V.band.data(), V.band.size() * sizeof(uint16_t),
                           hipMemcpyHostToDevice));
      HIP_TRY(c, hipMemcpy(c->ws + V.off_band_dirs, V.band_dirs.data(), V.band_dirs.size() * sizeof(uint32_t),
                           hipMemcpyHostToDevice));
    }
    HIP_TRY(c, hipMemcpy(c->ws + V.off_band_off, V.band_off.data(), V.band_off.size() * sizeof(int),
                         hipMemcpyHostToDevice));
    V.n_int = (int)V.interior.size();
    V.n_ghost = (int)V.ghost.size();
    V.n_iface = (int)V.iface.size();
  }
  HIP_TRY(c, hipMemcpy(c->ws + f.off_leaf[f.leaf_tab], f.leaf.data(), f.leaf.size(), hipMemcpyHostToDevice));
  return VMLBM_OK;
}

// flags of every level: coalescence cells; particle mapping on the finest level
int mark_flags(vmlbm_ctx* c) {
  Forest& f = *c->forest;
  for (int l = 0; l <= f.L; ++l) {
    Forest::Lev& V = f.lv[l];
    HIP_TRY(c, hipMemsetAsync(c->ws + V.off_flags, 0, (size_t)V.cap * kBlockCells, c->stream));
    if (V.n_iface) {
      k_mark_iface<<<(V.n_iface + 255) / 256, 256, 0, c->stream>>>((uint8_t*)(c->ws + V.off_flags),
                                                                   (const IfaceEntry*)(c->ws + V.off_iface), V.n_iface);
      HIP_TRY(c, hipGetLastError());
    }
  }
  const int np = (int)c->spheres.size();
  if (np) {
    Forest::Lev& V = f.lv[f.L];
    k_map_level<<<V.n_int, 256, 0, c->stream>>>((uint8_t*)(c->ws + V.off_flags), (uint16_t*)(c->ws + f.off_owner),
                                                c->parts(), np, finest_params(c), finest_addr(c),
                                                (const int*)(c->ws + V.off_pos), c->status());
    HIP_TRY(c, hipGetLastError());
  }
  return VMLBM_OK;
}

// explosions of levels l .. L-1 into the next finer level, one launch
int explode_chain(vmlbm_ctx* c, int l) {
  Forest& f = *c->forest;
  ExplodeChain ch{};
  int total = 0;
  for (int k = l; k < f.L; ++k) {
    Forest::Lev& C = f.lv[k];
    Forest::Lev& F = f.lv[k + 1];
    if (!F.n_ghost) continue;
    ExplodeSet& e = ch.set[ch.n++];
    e.coarse = c->ws + C.off_pdf[C.cur];
    e.fine = c->ws + F.off_pdf[F.cur];
    e.ex = (const int*)(c->ws + F.off_explode);
    e.band_off = (const int*)(c->ws + F.off_band_off);
    e.band = (const uint16_t*)(c->ws + F.off_band);
    e.dirs = (const uint32_t*)(c->ws + F.off_band_dirs);
    e.first = total;
    total += F.n_ghost;
  }
  if (!total) return VMLBM_OK;
  return dispatch(c->cfg.storage, [&](auto* tag) -> int {
    using S = std::remove_pointer_t<decltype(tag)>;
    k_explode<S><<<dim3(total, kBandSplit), 256, 0, c->stream>>>(ch);
    HIP_TRY(c, hipGetLastError());
    return VMLBM_OK;
  });
}

// the main stream waits for a particle update left on the side stream
int join_side(vmlbm_ctx* c) {
  Forest& f = *c->forest;
  if (!f.side_pending) return VMLBM_OK;
  HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
  f.side_pending = false;
  return VMLBM_OK;
}

// one sweep of level l (sub: its sub-step within the coarser level's step):
// interior blocks, coalescence cells and ghost bands in one launch
int launch_level(vmlbm_ctx* c, int l, int sub, const LevelArgs& a) {
  Forest& f = *c->forest;
  Forest::Lev& V = f.lv[l];
  LevelRoles r{};
  r.n_sweep = (uint32_t)V.n_int * kBlock;
  if (V.n_iface) {
    r.n_iface = V.n_iface;
    r.n_iface_wg = (V.n_iface + kIfaceCells - 1) / kIfaceCells;
    r.fine = c->ws + f.lv[l + 1].off_pdf[f.lv[l + 1].cur];
    r.iface = (const IfaceEntry*)(c->ws + V.off_iface);
  }
  r.n_ghost_wg = V.n_ghost * kBandSplit;
  r.ghost = (const int*)(c->ws + V.off_ghost);
  r.band_off = (const int*)(c->ws + V.off_band_off);
  r.band = (const uint16_t*)(c->ws + V.off_band);
  r.dirs = (const uint32_t*)(c->ws + V.off_band_dirs) + 1 + sub;
  r.n_lead = ((uint32_t)(r.n_ghost_wg + r.n_iface_wg) + 7u) & ~7u;
  const uint32_t grid = r.n_lead + r.n_sweep;
  if (!grid) return VMLBM_OK;
  const void* src = c->ws + V.off_pdf[V.cur];
  void* dst = c->ws + V.off_pdf[1 - V.cur];
  return dispatch(c->cfg.storage, [&](auto* tag) -> int {
    using S = std::remove_pointer_t<decltype(tag)>;
    const uint8_t* flags = (const uint8_t*)(c->ws + V.off_flags);
    const int* list = (const int*)(c->ws + V.off_int);
    if (a.sb != a.sp)
      k_level<S, true><<<grid, 256, 0, c->stream>>>((const S*)src, (S*)dst, flags, list, c->status(), a, r);
    else
      k_level<S, false><<<grid, 256, 0, c->stream>>>((const S*)src, (S*)dst, flags, list, c->status(), a, r);
    HIP_TRY(c, hipGetLastError());
    return VMLBM_OK;
  });
}

// link cells of the finest level, found per workgroup in its share of each
// sphere's box
int launch_link_cells(vmlbm_ctx* c, const SweepParams& p, const void* src, void* dst) {
  Forest& f = *c->forest;
  Forest::Lev& V = f.lv[f.L];
  const int np = (int)c->spheres.size();
  return dispatch(c->cfg.storage, [&](auto* tag) -> int {
    using S = std::remove_pointer_t<decltype(tag)>;
    k_link_cells<S, BAddr><<<dim3(link_chunks(p.box), np), dim3(256), 0, c->stream>>>(
        (const S*)src, (S*)dst, (const uint8_t*)(c->ws + V.off_flags), (const uint16_t*)(c->ws + f.off_owner),
        c->parts(), c->slots(), c->status(), p, finest_addr(c));
    HIP_TRY(c, hipGetLastError());
    return VMLBM_OK;
  });
}

// sub: 0 or 1, the first or second step of level l within a level-(l-1) step
int sweep_level(vmlbm_ctx* c, int l, int sub) {
  Forest& f = *c->forest;
  const int np = (int)c->spheres.size();
  const bool parts_here = l == f.L && np > 0;
  if (parts_here) {
    int rj = join_side(c);
    if (rj) return rj;
  }
  Forest::Lev& V = f.lv[l];
  const LevelArgs a = level_args(c, l, V.tab);
  void* src = c->ws + V.off_pdf[V.cur];
  void* dst = c->ws + V.off_pdf[1 - V.cur];
  int rc = launch_level(c, l, sub, a);
  if (rc) return rc;
  const SweepParams p = parts_here ? finest_params(c) : SweepParams{};
  if (parts_here) {
    rc = launch_link_cells(c, p, src, dst);
    if (rc) return rc;
  }
  V.cur = 1 - V.cur;
  c->cell_updates += (double)V.n_int * kBlockCells;
  if (parts_here) {
    // After the second of two finest steps the coarser level's sweep comes
    // next and touches no particle data, so the particle update (reduction,
    // re-mapping and refill) runs beside it on the side stream; the next
    // finest step, the end of the coarse step and the layout check join it.
    // (Measured on the 3-level workload: 2 % faster in FP32 than one stream;
    // the link cells beside the sweep and the coarsest sweep beside the finer
    // levels gained nothing, the cross-stream waits cost what they saved.)
    hipStream_t ps = c->stream;
    if (sub == 1 && f.L > 0) {
      HIP_TRY(c, hipEventRecord(c->ev_fork, c->stream));
      HIP_TRY(c, hipStreamWaitEvent(c->side, c->ev_fork, 0));
      ps = c->side;
    }
    HIP_TRY(c, launch_reduce_update(c->parts(), np, c->slots(), c->hist(), c->status(), p,
                                    update_params(c, c->fine_steps_done), ps));
    if (c->moving) {
      // re-mapping and refill change flags and populations of the new state
      rc = dispatch(c->cfg.storage, [&](auto* tag) -> int {
        using S = std::remove_pointer_t<decltype(tag)>;
        const int rb = p.box + 1;
        dim3 grid(2 * ((rb * rb * rb + 255) / 256), np), block(256);
        k_refill_remap<S, BAddr><<<grid, block, 0, ps>>>((S*)(c->ws + V.off_pdf[V.cur]),
                                                         (uint8_t*)(c->ws + V.off_flags),
                                                         (uint16_t*)(c->ws + f.off_owner), c->parts(), np, p,
                                                         finest_addr(c), c->status());
        HIP_TRY(c, hipGetLastError());
        return VMLBM_OK;
      });
      if (rc) return rc;
    }
    if (ps != c->stream) {
      HIP_TRY(c, hipEventRecord(c->ev_join, c->side));
      f.side_pending = true;
    }
  }
  if (l == f.L) c->fine_steps_done += 1;
  return VMLBM_OK;
}

// exploded: the explosion of level l (into l + 1) has already run, in the
// launch of the coarser level's step that also covered it
int step_level(vmlbm_ctx* c, int l, int sub, bool exploded = false) {
  Forest& f = *c->forest;
  if (l < f.L) {
    int rc = exploded ? VMLBM_OK : explode_chain(c, l);
    if (rc) return rc;
    rc = step_level(c, l + 1, 0, true);
    if (rc) return rc;
    rc = step_level(c, l + 1, 1);
    if (rc) return rc;
  }
  return sweep_level(c, l, sub);
}

// re-check the layout around the particles; move data if it changed
// Curl-sensor targets (Sec. 4.2.2): each leaf block's sensor, one level up
// above sigma_c, one down below c sigma_c, raised into t (finest block
// positions)
int flow_targets(vmlbm_ctx* c, std::vector<int8_t>& t) {
  Forest& f = *c->forest;
  const double sig = c->cfg.curl_threshold, csig = c->cfg.curl_coarsen * sig;
  for (int l = 0; l <= f.L; ++l) {
    Forest::Lev& V = f.lv[l];
    if (!V.n_int) continue;
    const LevelArgs a = level_args(c, l, V.tab);
    double* vel = (double*)(c->ws + V.off_vel);
    double* sens = (double*)(c->ws + V.off_sens);
    int rc = dispatch(c->cfg.storage, [&](auto* tag) -> int {
      using S = std::remove_pointer_t<decltype(tag)>;
      k_level_velocity<S><<<V.n_int, 256, 0, c->stream>>>((const S*)(c->ws + V.off_pdf[V.cur]),
                                                          (const int*)(c->ws + V.off_int), a, vel);
      HIP_TRY(c, hipGetLastError());
      return VMLBM_OK;
    });
    if (rc) return rc;
    const double s = (double)(1 << (f.L - l));
    const uint8_t* fl = (l == f.L && !c->spheres.empty()) ? (const uint8_t*)(c->ws + V.off_flags) : nullptr;
    k_block_curl<<<V.n_int, 256, 0, c->stream>>>(vel, fl, (const int*)(c->ws + V.off_int), V.n_int, a,
                                                 s * std::sqrt(s) / (2.0 * s), sens);
    HIP_TRY(c, hipGetLastError());
    std::vector<double> hs(V.n_int);
    HIP_TRY(c, hipMemcpyAsync(hs.data(), sens, V.n_int * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int sh = f.L - l, e = 1 << sh;
    for (int i = 0; i < V.n_int; ++i) {
      const int slot = V.interior[i];
      const double v = hs[slot];
      const int want = v > sig ? std::min(l + 1, f.L) : (v < csig ? std::max(l - 1, 0) : l);
      const int bi = V.pos[3 * slot], bj = V.pos[3 * slot + 1], bk = V.pos[3 * slot + 2];
      for (int z = 0; z < e; ++z)
        for (int y = 0; y < e; ++y)
          for (int x = 0; x < e; ++x) {
            int8_t& tv = t[f.lpos((bi << sh) + x, (bj << sh) + y, (bk << sh) + z)];
            tv = std::max<int8_t>(tv, (int8_t)want);
          }
    }
  }
  return VMLBM_OK;
}

// The layout changes when a sphere's block range does, and the new tables
// depend on nothing but the new ranges (and the static regions).  After a
// check, the ranges of the next change are predicted by carrying the
// spheres on at their current velocities (the first of the next
// kPredictChecks checks at which a range differs), and the tables for them
// are built on a host thread while the device steps.  A check that finds
// those ranges takes the tables instead of building them; any other change
// builds as before.  Not with the curl sensor, whose targets depend on the
// flow.
constexpr int kPredictChecks = 4096;

std::vector<int> predicted_boxes(const vmlbm_ctx* c, const Forest& f, const std::vector<vmlbm_sphere>& sph,
                                 const DevParticle* hp) {
  const double b = kBlock, dt = (double)c->cfg.check_every * (double)(1 << f.L);
  // earliest check at which some range may change: a face of a range
  // (centre -/+ (r + b)) reaches the next block boundary
  double kmin = kPredictChecks + 1;
  for (size_t i = 0; i < sph.size(); ++i)
    for (int a = 0; a < 3; ++a) {
      const double v = hp[i].u[a] * dt;
      if (!(std::fabs(v) > 0.0)) continue;
      const double lo = sph[i].x[a] - sph[i].radius - b, hi = sph[i].x[a] + sph[i].radius + b;
      const double d = v > 0 ? std::min((std::floor(lo / b) + 1) * b - lo, (std::floor(hi / b) + 1) * b - hi)
                             : std::min(lo - std::floor(lo / b) * b, hi - std::ceil(hi / b - 1) * b);
      kmin = std::min(kmin, d / std::fabs(v));
    }
  std::vector<vmlbm_sphere> s = sph;
  for (int k = std::max(1, (int)kmin - 1); k <= kPredictChecks && k <= (int)kmin + 2; ++k) {
    for (size_t i = 0; i < sph.size(); ++i)
      for (int a = 0; a < 3; ++a) s[i].x[a] = sph[i].x[a] + hp[i].u[a] * dt * k;
    std::vector<int> nb = sphere_boxes(s);
    if (nb != f.boxes) return nb;
  }
  return {};
}

void prebuild_next(vmlbm_ctx* c, Forest& f, const std::vector<vmlbm_sphere>& sph) {
  if (f.flow || sph.empty() || !f.host_parts) return;
  std::vector<int> nb = predicted_boxes(c, f, sph, f.host_parts);
  if (nb.empty() || (f.pre && f.pre->box == nb)) return;
  if (f.job.joinable()) f.job.join();   // one build at a time
  auto p = std::make_shared<Forest::Prebuilt>();
  p->box = nb;
  // the build runs on a skeleton forest of its own: geometry, capacities
  // and the targets of the predicted ranges
  auto g = std::make_shared<Forest>();
  g->L = f.L;
  for (int a = 0; a < 3; ++a) { g->nb0[a] = f.nb0[a]; g->nbL[a] = f.nbL[a]; }
  g->lv.resize(f.lv.size());
  for (size_t l = 0; l < f.lv.size(); ++l) {
    Forest::Lev& G = g->lv[l];
    const Forest::Lev& V = f.lv[l];
    for (int a = 0; a < 3; ++a) { G.n[a] = V.n[a]; G.nb[a] = V.nb[a]; }
    G.npos = V.npos;
    G.cap = V.cap;
    G.iface_cap = V.iface_cap;
  }
  std::vector<int8_t> t = layout_targets(f, nb);
  f.pre = p;
  f.job = std::thread([p, g, t]() {
    // a failed build (capacity, memory) is left to the check, which then
    // builds at the check and reports the error itself
    try {
      g->leaf = balance_layout(*g, t);
      p->rc = build_tables(nullptr, *g);
      p->leaf = std::move(g->leaf);
      p->lv = std::move(g->lv);
    } catch (...) {
      p->rc = VMLBM_ENOMEM;
    }
  });
}

int check_layout(vmlbm_ctx* c) {
  Forest& f = *c->forest;
  const int np = (int)c->spheres.size();
  std::vector<vmlbm_sphere> sph = c->spheres;
  // the positions come back by one copy on the stream into pinned memory,
  // queued behind the step, and one synchronisation
  if (np && !f.host_parts)
    HIP_TRY(c, hipHostMalloc((void**)&f.host_parts, np * sizeof(DevParticle), hipHostMallocDefault));
  if (np)
    HIP_TRY(c, hipMemcpyAsync(f.host_parts, c->parts(), np * sizeof(DevParticle), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < np; ++i)
    for (int a = 0; a < 3; ++a) sph[i].x[a] = f.host_parts[i].x[a];
  std::vector<int> box = sphere_boxes(sph);
  if (box == f.boxes && !f.flow) {
    prebuild_next(c, f, sph);
    return VMLBM_OK;
  }
  std::shared_ptr<Forest::Prebuilt> hit;
  if (!f.flow && f.pre && f.pre->box == box) {
    if (f.job.joinable()) f.job.join();
    if (f.pre->rc == VMLBM_OK) hit = f.pre;
    f.pre.reset();
  }
  std::vector<int8_t> nl;
  if (hit) {
    nl = std::move(hit->leaf);
  } else {
    std::vector<int8_t> t = layout_targets(f, box);
    if (f.flow) {
      int rc = flow_targets(c, t);
      if (rc) return rc;
    }
    nl = balance_layout(f, t);
  }
  if (nl == f.leaf) {
    f.boxes = box;
    prebuild_next(c, f, sph);
    return VMLBM_OK;
  }
  // the old layout stays readable on the device: leaf array, slot_of tables
  // and populations of the current buffers
  MigrateArgs m{};
  m.L = f.L;
  m.seed = kMigrateSeed + (uint32_t)f.refinements;
  for (int a = 0; a < 3; ++a) m.nbL[a] = f.nbL[a];
  m.old_leaf = (const int8_t*)(c->ws + f.off_leaf[f.leaf_tab]);
  for (int l = 0; l <= f.L; ++l) {
    Forest::Lev& V = f.lv[l];
    m.old_pdf[l] = c->ws + V.off_pdf[V.cur];
    m.old_slot_of[l] = (const int*)(c->ws + V.off_slot_of[V.tab]);
    for (int a = 0; a < 3; ++a) m.nb[l][a] = V.nb[a];
  }
  std::vector<int8_t> old = f.leaf;
  f.leaf = nl;
  int rc = VMLBM_OK;
  if (hit) {
    for (int l = 0; l <= f.L; ++l) {
      Forest::Lev& V = f.lv[l];
      Forest::Lev& H = hit->lv[l];
      V.slot_of = std::move(H.slot_of);
      V.interior = std::move(H.interior);
      V.ghost = std::move(H.ghost);
      V.pos = std::move(H.pos);
      V.nbr = std::move(H.nbr);
      V.explode = std::move(H.explode);
      V.band = std::move(H.band);
      V.band_off = std::move(H.band_off);
      V.band_dirs = std::move(H.band_dirs);
      V.iface = std::move(H.iface);
    }
    f.prebuilt_taken += 1;
  } else {
    rc = build_tables(c, f);
    if (rc) { f.leaf = old; return rc; }
  }
  for (int l = 0; l <= f.L; ++l) f.lv[l].tab = 1 - f.lv[l].tab;
  f.leaf_tab = 1 - f.leaf_tab;
  rc = upload_tables(c);
  if (rc) return rc;
  rc = dispatch(c->cfg.storage, [&](auto* tag) -> int {
    using S = std::remove_pointer_t<decltype(tag)>;
    for (int l = 0; l <= f.L; ++l) {
      Forest::Lev& V = f.lv[l];
      if (!V.n_int) continue;
      k_migrate<S><<<V.n_int, 256, 0, c->stream>>>((S*)(c->ws + V.off_pdf[1 - V.cur]), (const int*)(c->ws + V.off_int),
                                                   (const int*)(c->ws + V.off_pos), l, m,
                                                   c->status());
      HIP_TRY(c, hipGetLastError());
    }
    return VMLBM_OK;
  });
  if (rc) return rc;
  for (int l = 0; l <= f.L; ++l) f.lv[l].cur = 1 - f.lv[l].cur;
  rc = mark_flags(c);
  if (rc) return rc;
  f.boxes = box;
  f.refinements += 1;
  prebuild_next(c, f, sph);
  return VMLBM_OK;
}

}  // namespace

int refine_create(vmlbm_ctx* c) {
  const vmlbm_config& g = c->cfg;
  if (g.block != kBlock) return fail(c, VMLBM_EINVAL, "block edge must be %d", kBlock);
  if (g.levels < 1 || g.levels > kMaxLevels) return fail(c, VMLBM_EINVAL, "levels must lie in 1..%d", kMaxLevels);
  for (int a = 0; a < 3; ++a) {
    if (!g.periodic[a]) return fail(c, VMLBM_EINVAL, "the refined grid is periodic");
    if (g.n[a] % kBlock) return fail(c, VMLBM_EINVAL, "coarse cells must be a multiple of %d", kBlock);
  }
  auto* f = new Forest();
  f->L = g.levels - 1;
  for (int a = 0; a < 3; ++a) {
    f->nb0[a] = g.n[a] / kBlock;
    f->nbL[a] = f->nb0[a] << f->L;
  }
  const long NB = (long)f->nbL[0] * f->nbL[1] * f->nbL[2];
  if (NB > (1L << 26)) { delete f; return fail(c, VMLBM_ERANGE, "too many finest block positions"); }
  f->base.assign(NB, 0);
  f->flow = g.curl_threshold > 0.0;
  f->lv.resize(f->L + 1);
  double tau = 1.0 / g.omega;
  for (int l = f->L; l >= 0; --l) {
    Forest::Lev& V = f->lv[l];
    for (int a = 0; a < 3; ++a) {
      V.n[a] = g.n[a] << l;
      V.nb[a] = f->nb0[a] << l;
    }
    V.npos = (long)V.nb[0] * V.nb[1] * V.nb[2];
    V.lp.sp = 1.0 / tau;
    V.lp.sm = s_minus_of(V.lp.sp, g.magic);
    V.lp.sb = s_bulk_of(V.lp.sp, g.bulk_factor);
    for (int a = 0; a < 3; ++a) V.lp.F[a] = g.body_force[a] * (double)(1 << (f->L - l));
    tau = 0.5 + 0.5 * (tau - 0.5);
  }
  c->forest = std::unique_ptr<Forest, void (*)(Forest*)>(f, forest_free);
  return VMLBM_OK;
}

int refine_plan(vmlbm_ctx* c) {
  Forest& f = *c->forest;
  // layout from the spheres' initial positions and the static regions
  f.boxes = sphere_boxes(c->spheres);
  f.leaf = balance_layout(f, layout_targets(f, f.boxes));
  for (auto& V : f.lv) { V.cap = 0; V.iface_cap = 0; }
  int rc = build_tables(c, f);
  if (rc) return rc;
  std::vector<long> cap, icap;
  plan_capacity(c, f, cap, icap);
  const size_t S = storage_bytes(c->cfg.storage);
  int box = 0;
  for (const auto& s : c->spheres) box = std::max(box, (int)std::ceil(2.0 * s.radius) + 7);
  c->box = box;
  // one force slot per workgroup of the link-cell pass (a box share each)
  c->slot_stride = (size_t)link_chunks(box) * kSlotWords;
  const int np = (int)c->spheres.size();
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = (off + bytes + 255) & ~size_t(255); return o; };
  c->off_status = take(kStatusWords * sizeof(int));
  c->off_parts = take(std::max(np, 1) * sizeof(DevParticle));
  c->off_slots = take(std::max<size_t>(np * c->slot_stride, 1) * sizeof(double));
  c->off_hist = take((size_t)std::max(c->cfg.history, 1) * std::max(np, 1) * kHistWords * sizeof(double));
  c->off_totals = take((size_t)kTotalsGroups * 8 * sizeof(double));
  for (int l = 0; l <= f.L; ++l) {
    Forest::Lev& V = f.lv[l];
    V.cap = (int)std::max<long>(cap[l], (long)(V.pos.size() / 3));
    V.iface_cap = (int)std::max<long>(icap[l], (long)V.iface.size());
    for (int b = 0; b < 2; ++b) V.off_pdf[b] = take((size_t)kQ * V.cap * kBlockCells * S);
    V.off_flags = take((size_t)V.cap * kBlockCells);
    for (int b = 0; b < 2; ++b) V.off_slot_of[b] = take(V.npos * sizeof(int));
    V.off_pos = take((size_t)V.cap * 3 * sizeof(int));
    V.off_nbr = take((size_t)V.cap * kNbrWords * sizeof(int));
    V.off_int = take((size_t)V.cap * sizeof(int));
    V.off_ghost = take((size_t)V.cap * sizeof(int));
    V.off_explode = take((size_t)V.cap * 5 * sizeof(int));
    V.off_iface = take((size_t)V.iface_cap * sizeof(IfaceEntry));
    V.off_band = take((size_t)V.cap * kBlockCells * sizeof(uint16_t));
    V.off_band_off = take((size_t)(V.cap + 1) * sizeof(int));
    V.off_band_dirs = take((size_t)V.cap * kBlockCells * 3 * sizeof(uint32_t));
    if (f.flow) {
      V.off_vel = take((size_t)3 * V.cap * kBlockCells * sizeof(double));
      V.off_sens = take((size_t)V.cap * sizeof(double));
    }
  }
  f.off_owner = take((size_t)f.lv[f.L].cap * kBlockCells * sizeof(uint16_t));
  for (int b = 0; b < 2; ++b) f.off_leaf[b] = take(f.leaf.size());
  c->ws_needed = off;
  return VMLBM_OK;
}

int refine_init(vmlbm_ctx* c, double rho, const double* u0) {
  Forest& f = *c->forest;
  const int np = (int)c->spheres.size();
  f.boxes = sphere_boxes(c->spheres);
  f.leaf = balance_layout(f, layout_targets(f, f.boxes));
  int rc = build_tables(c, f);
  if (rc) return rc;
  for (auto& V : f.lv) { V.tab = 0; V.cur = 0; }
  f.leaf_tab = 0;
  rc = upload_tables(c);
  if (rc) return rc;
  HIP_TRY(c, hipMemsetAsync(c->status(), 0, kStatusWords * sizeof(int), c->stream));
  std::vector<DevParticle> hp(np);
  for (int i = 0; i < np; ++i) {
    const vmlbm_sphere& s = c->spheres[i];
    DevParticle& P = hp[i];
    memset(&P, 0, sizeof(P));
    for (int a = 0; a < 3; ++a) {
      P.x[a] = s.x[a];
      P.xold[a] = s.x[a];
      P.u[a] = s.fixed ? 0.0 : s.u[a];
      P.w[a] = s.fixed == 1 ? 0.0 : s.w[a];
    }
    P.r = s.radius; P.rho = s.density_ratio; P.cv = s.cv; P.cvw = s.cv_omega;
    P.fixed = s.fixed;
    P.scheme = s.vm_scheme; P.nvel = 1;
    for (int a = 0; a < 3; ++a) {
      const int n = f.lv[f.L].n[a];
      int lo = (int)std::floor(s.x[a] - s.radius) - 3;
      lo = ((lo % n) + n) % n;
      P.box_lo[a] = lo;
      P.remap_lo[a] = lo;
    }
  }
  if (np) HIP_TRY(c, hipMemcpyAsync(c->parts(), hp.data(), np * sizeof(DevParticle), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->hist(), 0, (size_t)c->cfg.history * std::max(np, 1) * kHistWords * sizeof(double), c->stream));
  // velocity staging in the second buffer of level 0
  Forest::Lev& V0 = f.lv[0];
  const uint32_t N0 = (uint32_t)((size_t)c->cfg.n[0] * c->cfg.n[1] * c->cfg.n[2]);
  double* u0d = nullptr;
  if (u0) {
    const size_t need = 3 * (size_t)N0 * sizeof(double);
    if (need > (size_t)kQ * V0.cap * kBlockCells * storage_bytes(c->cfg.storage))
      return fail(c, VMLBM_ERANGE, "velocity staging does not fit");
    u0d = (double*)(c->ws + V0.off_pdf[1]);
    HIP_TRY(c, hipMemcpyAsync(u0d, u0, need, hipMemcpyHostToDevice, c->stream));
  }
  rc = dispatch(c->cfg.storage, [&](auto* tag) -> int {
    using S = std::remove_pointer_t<decltype(tag)>;
    for (int l = 0; l <= f.L; ++l) {
      Forest::Lev& V = f.lv[l];
      const int ns = V.n_int + V.n_ghost;
      if (!ns) continue;
      LevelArgs ai = level_args(c, l, 0);
      ai.seed = kInitSeed + (uint32_t)l;
      k_init_level<S><<<ns, 256, 0, c->stream>>>((S*)(c->ws + V.off_pdf[0]), u0d, l, c->cfg.n[0], c->cfg.n[1], N0,
                                                 rho - 1.0, ai);
      HIP_TRY(c, hipGetLastError());
    }
    return VMLBM_OK;
  });
  if (rc) return rc;
  rc = mark_flags(c);
  if (rc) return rc;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->steps_done = 0;
  c->fine_steps_done = 0;
  f.refinements = 0;
  f.prebuilt_taken = 0;
  f.coarse_steps = 0;
  c->cur = 0;
  c->initialized = true;
  return VMLBM_OK;
}

int refine_step(vmlbm_ctx* c, int n) {
  Forest& f = *c->forest;
  for (int s = 0; s < n; ++s) {
    int rc = step_level(c, 0, 0);
    const int rj = join_side(c);
    if (rc) return rc;
    if (rj) return rj;
    c->steps_done += 1;
    f.coarse_steps += 1;
    if (c->cfg.check_every > 0 && f.coarse_steps % c->cfg.check_every == 0) {
      rc = check_layout(c);
      if (rc) return rc;
    }
  }
  return VMLBM_OK;
}

int refine_level_cells(vmlbm_ctx* c, int level, size_t* cells) {
  Forest& f = *c->forest;
  if (level < 0 || level > f.L) return fail(c, VMLBM_EINVAL, "bad level");
  *cells = (size_t)f.lv[level].n_int * kBlockCells;
  return VMLBM_OK;
}

static int read_level_raw(vmlbm_ctx* c, int level, std::vector<double>& out, std::vector<uint8_t>& fl) {
  Forest& f = *c->forest;
  Forest::Lev& V = f.lv[level];
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const size_t S = storage_bytes(c->cfg.storage);
  const size_t cells = (size_t)V.n_int * kBlockCells;
  out.assign(kQ * cells, 0.0);
  fl.assign(cells, 0);
  std::vector<char> raw(kQ * cells * S);
  // interior slots are 0..n_int-1, contiguous at the front of the pool
  HIP_TRY(c, hipMemcpy(raw.data(), c->ws + V.off_pdf[V.cur], kQ * cells * S, hipMemcpyDeviceToHost));
  for (int q = 0; q < kQ; ++q)
    for (size_t i = 0; i < cells; ++i) {
      const size_t k = bpop(q, (uint32_t)i);
      double d;
      if (c->cfg.storage == VMLBM_F64) d = ((const double*)raw.data())[k];
      else if (c->cfg.storage == VMLBM_F32) d = ((const float*)raw.data())[k];
      else d = __half2float(((const __half*)raw.data())[k]);
      out[q * cells + i] = w_of(q) + d;
    }
  HIP_TRY(c, hipMemcpy(fl.data(), c->ws + V.off_flags, cells, hipMemcpyDeviceToHost));
  return VMLBM_OK;
}

int refine_read_populations(vmlbm_ctx* c, int level, double* out) {
  Forest& f = *c->forest;
  if (level < 0 || level > f.L) return fail(c, VMLBM_EINVAL, "bad level");
  std::vector<double> v;
  std::vector<uint8_t> fl;
  int rc = read_level_raw(c, level, v, fl);
  if (rc) return rc;
  const size_t cells = fl.size();
  for (int q = 0; q < kQ; ++q)
    for (size_t i = 0; i < cells; ++i) out[q * cells + i] = (fl[i] & kSolid) ? 0.0 : v[q * cells + i];
  return VMLBM_OK;
}

int refine_write_populations(vmlbm_ctx* c, int level, const double* in) {
  Forest& f = *c->forest;
  if (level < 0 || level > f.L) return fail(c, VMLBM_EINVAL, "bad level");
  Forest::Lev& V = f.lv[level];
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const size_t S = storage_bytes(c->cfg.storage);
  const size_t cells = (size_t)V.n_int * kBlockCells;
  std::vector<char> raw(kQ * cells * S);
  for (int q = 0; q < kQ; ++q)
    for (size_t i = 0; i < cells; ++i) {
      const size_t k = bpop(q, (uint32_t)i);
      const double d = in[q * cells + i] - w_of(q);
      if (c->cfg.storage == VMLBM_F64) ((double*)raw.data())[k] = d;
      else if (c->cfg.storage == VMLBM_F32) ((float*)raw.data())[k] = (float)d;
      else ((uint16_t*)raw.data())[k] = half_bits_rne(d);
    }
  HIP_TRY(c, hipMemcpy(c->ws + V.off_pdf[V.cur], raw.data(), kQ * cells * S, hipMemcpyHostToDevice));
  return VMLBM_OK;
}

int refine_read_owner(vmlbm_ctx* c, int level, int* out) {
  Forest& f = *c->forest;
  if (level < 0 || level > f.L) return fail(c, VMLBM_EINVAL, "bad level");
  Forest::Lev& V = f.lv[level];
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const size_t cells = (size_t)V.n_int * kBlockCells;
  std::vector<uint8_t> fl(cells);
  std::vector<uint16_t> ow(cells, 0);
  HIP_TRY(c, hipMemcpy(fl.data(), c->ws + V.off_flags, cells, hipMemcpyDeviceToHost));
  if (level == f.L && !c->spheres.empty())
    HIP_TRY(c, hipMemcpy(ow.data(), c->ws + f.off_owner, cells * 2, hipMemcpyDeviceToHost));
  for (size_t i = 0; i < cells; ++i) out[i] = (fl[i] & kSolid) ? (int)ow[i] : -1;
  return VMLBM_OK;
}

int refine_cell_counts(vmlbm_ctx* c, int level, long long* fluid, long long* interior) {
  Forest& f = *c->forest;
  if (level < 0 || level > f.L) return fail(c, VMLBM_EINVAL, "bad level");
  Forest::Lev& V = f.lv[level];
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const size_t cells = (size_t)V.n_int * kBlockCells;
  std::vector<uint8_t> fl(cells);
  HIP_TRY(c, hipMemcpy(fl.data(), c->ws + V.off_flags, cells, hipMemcpyDeviceToHost));
  long long nf = 0, ni = 0;
  for (size_t i = 0; i < cells; ++i) { nf += !(fl[i] & kSolid); ni += fl[i] == 0; }
  if (fluid) *fluid = nf;
  if (interior) *interior = ni;
  return VMLBM_OK;
}

void refine_destroy(vmlbm_ctx*) {}

// volume-weighted totals over the interior fluid cells of every level;
// part: device partials (kTotalsGroups x 8 doubles), h: host buffer of the
// same size
int refine_totals(vmlbm_ctx* c, double* part, double* h, double* mass, double mom[3]) {
  Forest& f = *c->forest;
  long double m = 0, j[3] = {0, 0, 0};
  for (int l = 0; l <= f.L; ++l) {
    Forest::Lev& V = f.lv[l];
    if (!V.n_int) continue;
    HIP_TRY(c, launch_totals(c->cfg.storage, c->ws + V.off_pdf[V.cur], (const uint8_t*)(c->ws + V.off_flags),
                             PopLayout{}, 0, (const int*)(c->ws + V.off_int), V.n_int, part, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(h, part, (size_t)kTotalsGroups * 8 * sizeof(double), hipMemcpyDeviceToHost));
    long double n = 0, ml = 0, jl[3] = {0, 0, 0};
    for (int g = 0; g < kTotalsGroups; ++g) {
      n += h[8 * g]; ml += h[8 * g + 1];
      for (int a = 0; a < 3; ++a) jl[a] += h[8 * g + 2 + a];
    }
    const long double vol = 1.0L / (long double)(1L << (3 * l));
    m += (n + ml) * vol;
    for (int a = 0; a < 3; ++a) j[a] += jl[a] * vol;
  }
  if (mass) *mass = (double)m;
  if (mom) for (int a = 0; a < 3; ++a) mom[a] = (double)j[a];
  return VMLBM_OK;
}

void level_force(const vmlbm_ctx* c, int level, double F[3]) {
  const int L = c->cfg.block > 0 ? c->cfg.levels - 1 : 0;
  const double s = (double)(1 << (L - level));
  for (int a = 0; a < 3; ++a) F[a] = c->F[a] * s;
}

int refine_add_region(vmlbm_ctx* c, const int lo[3], const int hi[3], int level) {
  Forest& f = *c->forest;
  if (level < 0 || level > f.L) return fail(c, VMLBM_EINVAL, "bad level");
  const int s = 1 << f.L;
  for (int k = 0; k < f.nbL[2]; ++k)
    for (int j = 0; j < f.nbL[1]; ++j)
      for (int i = 0; i < f.nbL[0]; ++i) {
        const int p[3] = {i, j, k};
        bool in = true;
        for (int a = 0; a < 3; ++a) {
          const double b0 = (double)p[a] * kBlock / s, b1 = (double)(p[a] + 1) * kBlock / s;
          if (!(b1 > lo[a] && b0 < hi[a])) in = false;
        }
        if (in) f.base[f.lpos(i, j, k)] = (int8_t)std::max<int>(f.base[f.lpos(i, j, k)], level);
      }
  return VMLBM_OK;
}

// the level's pull without arithmetic (k_level_pull) `reps` times, each
// making the pulled state current
int refine_level_pull(vmlbm_ctx* c, int l, int reps) {
  Forest& f = *c->forest;
  int rc = join_side(c);
  if (rc) return rc;
  Forest::Lev& V = f.lv[l];
  const uint32_t n = (uint32_t)V.n_int * kBlock;
  const LevelArgs a = level_args(c, l, V.tab);
  for (int r = 0; r < reps; ++r) {
    if (n) {
      rc = dispatch(c->cfg.storage, [&](auto* tag) -> int {
        using S = std::remove_pointer_t<decltype(tag)>;
        k_level_pull<S><<<n, 256, 0, c->stream>>>((const S*)(c->ws + V.off_pdf[V.cur]), (S*)(c->ws + V.off_pdf[1 - V.cur]),
                                                  (const int*)(c->ws + V.off_int), a, n);
        HIP_TRY(c, hipGetLastError());
        return VMLBM_OK;
      });
      if (rc) return rc;
    }
    V.cur = 1 - V.cur;
  }
  return VMLBM_OK;
}

}  // namespace vm

using namespace vm;

extern "C" {

int vmlbm_add_refine_region(vmlbm_ctx* c, const int lo[3], const int hi[3], int level) {
  if (!c || !lo || !hi) return VMLBM_EINVAL;
  if (c->cfg.block <= 0 || !c->forest) return fail(c, VMLBM_ESTATE, "not a block-structured grid");
  if (c->ws) return fail(c, VMLBM_ESTATE, "regions must be added before the workspace is bound");
  return refine_add_region(c, lo, hi, level);
}

int vmlbm_level_blocks(vmlbm_ctx* c, int level, int* count, int* origin) {
  if (!c || !count) return VMLBM_EINVAL;
  if (c->cfg.block <= 0 || !c->forest) return fail(c, VMLBM_ESTATE, "not a block-structured grid");
  Forest& f = *c->forest;
  if (level < 0 || level > f.L) return fail(c, VMLBM_EINVAL, "bad level");
  const Forest::Lev& V = f.lv[level];
  *count = (int)V.interior.size();
  if (origin)
    for (size_t i = 0; i < V.interior.size(); ++i)
      for (int a = 0; a < 3; ++a) origin[3 * i + a] = V.pos[3 * V.interior[i] + a] * kBlock;
  return VMLBM_OK;
}

int vmlbm_refinements(vmlbm_ctx* c, int* count) {
  if (!c || !count) return VMLBM_EINVAL;
  *count = c->forest ? c->forest->refinements : 0;
  return VMLBM_OK;
}

int vmlbm_prebuilt_layouts(vmlbm_ctx* c, int* count) {
  if (!c || !count) return VMLBM_EINVAL;
  *count = c->forest ? c->forest->prebuilt_taken : 0;
  return VMLBM_OK;
}

int vmlbm_level_pull(vmlbm_ctx* c, int level, int reps) {
  if (!c) return VMLBM_EINVAL;
  if (c->cfg.block <= 0 || !c->forest) return fail(c, VMLBM_ESTATE, "not a block-structured grid");
  if (!c->ws) return fail(c, VMLBM_ESTATE, "workspace not bound");
  if (!c->initialized) return fail(c, VMLBM_ESTATE, "vmlbm_init_equilibrium not called");
  if (level < 0 || level > c->forest->L) return fail(c, VMLBM_EINVAL, "bad level");
  if (reps < 1) return fail(c, VMLBM_EINVAL, "reps must be at least 1");
  return refine_level_pull(c, level, reps);
}

}  // extern "C"
