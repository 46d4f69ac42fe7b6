// CPU check of the step kernel's index arithmetic: the LDS layout regions,
// the per-scene record block, and the bit fields of the packed keys, over
// the whole range of scene sizes and capacities the host accepts.  Built
// with g++ by tests/test_index_math.py (no GPU, no HIP runtime).
#define __host__
#define __device__
struct float4 {
  float x, y, z, w;
};
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2106_14405_amd/csrc/sim_internal.h"

using namespace rbs;

static int failures = 0;
#define CHECK(c, ...)                                   \
  do {                                                  \
    if (!(c)) {                                         \
      if (failures++ < 20) {                            \
        std::fprintf(stderr, "FAIL %s: ", #c);          \
        std::fprintf(stderr, __VA_ARGS__);              \
        std::fprintf(stderr, "\n");                     \
      }                                                 \
    }                                                   \
  } while (0)

struct Region {
  const char* name;
  long lo, hi;  // words [lo, hi)
};

static bool overlap(const Region& a, const Region& b) { return a.lo < b.hi && b.lo < a.hi; }

// regions that are live at the same time must be disjoint and inside [0, total)
static void disjoint(const std::vector<Region>& rs, long total, int NB, int PM, int CM, int W) {
  for (size_t i = 0; i < rs.size(); i++) {
    CHECK(rs[i].lo >= 0 && rs[i].hi <= total && rs[i].lo <= rs[i].hi, "%s [%ld,%ld) total %ld NB %d PM %d CM %d W %d",
          rs[i].name, rs[i].lo, rs[i].hi, total, NB, PM, CM, W);
    for (size_t j = i + 1; j < rs.size(); j++)
      CHECK(!overlap(rs[i], rs[j]), "%s and %s overlap NB %d PM %d CM %d W %d", rs[i].name, rs[j].name, NB, PM, CM, W);
  }
}

static void check_layout(int NB, int PM, int CM, int W, int solver, int warm, int arm) {
  const LdsLayout L = lds_layout(NB, PM, CM, W, solver, warm, arm);
  const long T = L.total;
  // resident for the whole step (the two slots in front of dyn and dyn2: ground and sink)
  std::vector<Region> res = {{"geo", L.geo, L.geo + 12L * NB},
                             {"dyn", L.dyn - 2L * kDynWords, L.dyn + (long)kDynWords * NB},
                             {"dyn2", L.dyn2 - 8, L.dyn2 + 4L * NB},
                             {"ckey", L.ckey, L.ckey + CM},
                             {"lam", L.lam, L.lam + 4L * CM},
                             {"perm", L.perm, L.perm + CM},
                             {"misc", L.misc, L.misc + kMiscWords},
                             {"hist", L.hist, L.hist + 256L * W},
                             {"hbase", L.hbase, L.hbase + 256},
                             {"scratch", L.scr, T}};
  if (warm == WARM_LEARNED) res.push_back({"fresh", L.fresh, L.fresh + (CM + 31) / 32});
  if ((arm & 3) == 2) res.push_back({"arm", L.arm, L.arm + kArmWords});
  if (arm & kArtParts) res.push_back({"parts", L.parts, L.parts + kPartWords});
  CHECK(((arm & 3) == 2) == (L.arm >= 0) && ((arm & kArtParts) != 0) == (L.parts >= 0), "arm/parts regions present");
  disjoint(res, T, NB, PM, CM, W);
  // a part's words inside its 16-word entry; the count word in front of the entries
  CHECK(PART_BODY < kPartStride && PART_KIND < kPartStride && PART_M < kPartStride && PART_BIAS + 2 <= PART_LAM &&
            PART_LAM + 2 <= PART_IM && PART_IM < PART_AX && PART_AX + 3 <= kPartStride &&
            kPartWords >= 4 + kMaxParts * kPartStride && kMaxParts <= 64,
        "part words");
  // the arm's words: M^-1, rates, impulses, targets, origins and axes inside the region
  CHECK(ARM_MI + 49 <= ARM_DQ && ARM_DQ + 7 <= ARM_QREF && ARM_QREF + 7 <= ARM_LAM && ARM_LAM + 7 <= ARM_BIAS &&
            ARM_BIAS + 7 <= ARM_O && ARM_O + 21 <= ARM_AX && ARM_AX + 21 <= kArmWords,
        "arm words");
  // misc slots: per-wave words and scan words fit
  CHECK(M_SCAN + W <= kMiscWords && M_WAVE + W <= M_SCAN, "misc slots");
  // colour starts (kMaxColours + 1) live in hbase; class bases 16, per-wave class counts 16 W in hist
  CHECK(kMaxColours + 1 <= 256 && 16 * W <= 256 * W, "hbase/hist sizes");
  // broadphase scratch
  disjoint({{"pk", L.pk, L.pk + PM},
            {"pk2", L.pk2, L.pk2 + PM},
            {"lo", L.lo, L.lo + 4L * NB},
            {"hi", L.hi, L.hi + 4L * NB},
            {"skey", L.skey, L.skey + NB},
            {"sval", L.sval, L.sval + NB},
            {"skey2", L.skey2, L.skey2 + NB},
            {"sval2", L.sval2, L.sval2 + NB}},
           T, NB, PM, CM, W);
  CHECK(L.pk >= L.scr, "pk in scratch");
  // narrowphase: the sorted pairs (pk or pk2) stay live beside the class
  // permutation and the per-pair counts (bytes)
  disjoint({{"pk", L.pk, L.pk + PM},
            {"pk2", L.pk2, L.pk2 + PM},
            {"nperm", L.nperm, L.nperm + PM},
            {"ncnt", L.ncnt, L.ncnt + (PM + 3) / 4}},
           T, NB, PM, CM, W);
  // colouring: previous keys (CM words) and colours (CM bytes) staged at deg
  // while colour is written; then lists
  disjoint({{"colour", L.colour, L.colour + CM}, {"pkeys+pcols", L.deg, L.deg + CM + (CM + 3) / 4}}, T, NB, PM, CM, W);
  disjoint({{"colour", L.colour, L.colour + CM},
            {"deg", L.deg, L.deg + NB + 1},
            {"lstart", L.lstart, L.lstart + NB + 1},
            {"list", L.list, L.list + 2L * CM},
            {"rank", L.rank, L.rank + CM}},
           T, NB, PM, CM, W);
  CHECK(L.colour >= L.scr, "colour in scratch");
  // colour sort copies (cv0, ck1 over the list) beside colour and rank
  disjoint({{"colour", L.colour, L.colour + CM},
            {"rank", L.rank, L.rank + CM},
            {"cv0", L.cv0, L.cv0 + CM},
            {"ck1", L.ck1, L.ck1 + CM}},
           T, NB, PM, CM, W);
  // solver: saved velocities, start objective terms, Jacobi snapshot and
  // increments beside colour and deg (both read later)
  std::vector<Region> sol = {{"colour", L.colour, L.colour + CM}, {"deg", L.deg, L.deg + NB + 1}};
  if (warm == WARM_LEARNED) {
    sol.push_back({"vsave", L.vsave, L.vsave + 8L * NB});
    sol.push_back({"fval", L.fval, L.fval + CM});
  }
  if (solver == SOLVER_JACOBI) {
    sol.push_back({"snap", L.snap, L.snap + 8L * NB});
    sol.push_back({"dl", L.dl, L.dl + 4L * CM});
  }
  disjoint(sol, T, NB, PM, CM, W);
  // outputs: arm force partial sums beside colour and deg
  disjoint({{"colour", L.colour, L.colour + CM}, {"deg", L.deg, L.deg + NB + 1}, {"force", L.force, L.force + CM}}, T,
           NB, PM, CM, W);
  // float4 alignment of the regions read as float4
  for (long o : {(long)L.geo, (long)L.dyn, (long)L.dyn2, (long)L.lam, (long)L.lo, (long)L.hi, (long)L.pk})
    CHECK(o % 4 == 0, "float4 alignment %ld", o);
}

int main() {
  // packed keys: pair key (a << 11) | b, b = 2047 the ground; contact key
  // (a << 20) | (b << 8) | feature, b = 0xFFF the ground; colour-major sort
  // key (colour << 16) | contact; list ranks packed as two 16-bit halves
  CHECK(kMaxBodiesPerScene <= 2047, "pair key body field (11 bits, 2047 = ground)");
  CHECK(kMaxBodiesPerScene <= 4095, "contact key body field (12 bits, 0xFFF = ground)");
  CHECK(kGroundKey == 0xFFFu && kGroundPair == 0xFFFFu, "ground codes");
  CHECK(kMaxColours <= 255, "colours stored in a byte");
  const int cm_max = kCapPerBody * kMaxBodiesPerScene;
  CHECK(cm_max <= 65535, "contact index in 16 bits (colour sort key, list ranks): %d", cm_max);
  // box-box features (ref bit | face << 1 | clip index << 4) and edge features (0x80 | 0..8) in 8 bits
  CHECK(((1 | (5 << 1) | (7 << 4)) & ~0xFF) == 0 && (0x80 | 8) <= 0xFF, "feature byte");

  const int NBs[] = {1, 2, 7, 8, 15, 16, 63, 64, 65, 100, 127, 128, 135, 255, 256, 511, 512, 513, 1000, 1023, 1024};
  const int capsB[] = {1, 2, 63, 64, 65, 384, 512, 513, 1024, 2048, 2560, 4096, 6144};
  long checked = 0;
  for (int NB : NBs) {
    if (NB > kMaxBodiesPerScene) continue;
    for (int PMb : capsB)
      for (int CMb : capsB) {
        // the capacities a scene of NB bodies gets from batch capacities PMb, CMb
        const int PM = scene_cap(NB, PMb), CM = scene_cap(NB, CMb);
        CHECK(PM <= PMb && CM <= CMb && PM >= 1 && CM >= 1, "scene_cap");
        // record block: 5 float4 per contact, or 4 staged contacts (2 float4 each) per pair
        const long rs = rec_stride(PMb, CMb);
        CHECK(8L * (PM - 1) + 2 * 3 + 1 < rs, "staging index inside the record block PM %d CM %d", PM, CM);
        CHECK((long)kRec * (CM - 1) + kRec - 1 < rs, "record index inside the record block");
        for (int W = 1; W <= 4; W++)
          for (int solver = 0; solver < 2; solver++)
            for (int warm = 0; warm < 3; warm++)
              for (int art : {0, 2, kArtParts, 2 | kArtParts}) {
                check_layout(NB, PM, CM, W, solver, warm, art);
                checked++;
              }
      }
  }
  std::printf("layouts checked: %ld, failures: %d\n", checked, failures);
  return failures ? 1 : 0;
}
