// Saving and restoring the temperature-independent state of a context: the
// electron and phonon tables and the vertex store B+/- of Eq. 8 (with the
// error codes of the GEMM forms), so that temperature and carrier sweeps
// can resume from a file instead of recomputing the vertices, as the
// method's workflow stores vertices and rates for reuse.
//
// File: magic "ELPHSAV1", a fixed header (sizes, parameters, a hash of the
// inputs), then the arrays (state k and band, energies, velocities, phonon
// energies and velocities, eigenvectors of the kept k, B+, B-, codes), then a
// hash of everything before it.  A file is loaded into a context created from
// the same inputs and parameters; the tables are rebuilt and must equal the
// saved ones bit for bit (same library and device), and the store is then
// taken from the file.
#include "common.h"
#include "tables.h"
#include "vertex.h"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

namespace elph {

namespace {

constexpr char kMagic[8] = {'E', 'L', 'P', 'H', 'S', 'A', 'V', '1'};
constexpr size_t kStage = (size_t)64 << 20;  // host staging block

struct SaveHeader {
  int32_t nb, na, nre, nrp, mesh[3], precision, delta, frohlich;
  double mu, window, sigma, omega_min;
  uint64_t input_hash;
  int64_t nk, nkept, nstates;
  int32_t store_f32, rho_valid, rho_stride, pad;
};

// 64-bit hash over 8-byte words (multiply-xor), then the tail bytes
struct Hasher {
  uint64_t h = 1469598103934665603ull;
  void add(const void* p, size_t n) {
    const unsigned char* c = (const unsigned char*)p;
    size_t k = 0;
    for (; k + 8 <= n; k += 8) {
      uint64_t w;
      std::memcpy(&w, c + k, 8);
      h = (h ^ w) * 1099511628211ull;
      h ^= h >> 29;
    }
    for (; k < n; ++k) h = (h ^ c[k]) * 1099511628211ull;
  }
};

// hash of device memory, staged through the host
static elph_status hash_device(elph_ctx ctx, const void* d, size_t bytes, Hasher* H, std::vector<char>& buf) {
  for (size_t o = 0; o < bytes; o += kStage) {
    const size_t n = std::min(kStage, bytes - o);
    HIPCHK(hipMemcpy(buf.data(), (const char*)d + o, n, hipMemcpyDeviceToHost));
    H->add(buf.data(), n);
  }
  return ELPH_OK;
}

static elph_status input_hash(elph_ctx ctx, uint64_t* out) {
  std::vector<char> buf(kStage);
  Hasher H;
  const int nb = ctx->nb, nbr = ctx->nbr;
  const size_t nn = (size_t)nb * nb, mm = (size_t)nbr * nbr;
  struct Arr {
    const void* p;
    size_t bytes;
  };
  const size_t nac = ctx->d_nac ? (size_t)ctx->na * 9 + 18 + (ctx->frohlich ? (size_t)ctx->na * 3 : 0) : 0;
  const Arr arrs[] = {
      {ctx->d_re, (size_t)ctx->nre * 3 * sizeof(int32_t)},
      {ctx->d_rp, (size_t)ctx->nrp * 3 * sizeof(int32_t)},
      {ctx->d_wre, ctx->d_wre ? (size_t)ctx->nre * sizeof(double) : 0},
      {ctx->d_wrp, ctx->d_wrp ? (size_t)ctx->nrp * sizeof(double) : 0},
      {ctx->d_hr, (size_t)ctx->nre * nn * 2 * sizeof(double)},
      {ctx->d_dr, (size_t)ctx->nrp * mm * sizeof(double)},
      {ctx->d_gr, (size_t)ctx->nre * ctx->nrp * nbr * nn * 2 * sizeof(double)},
      {ctx->d_mass_x, (size_t)nbr * sizeof(double)},
      {ctx->d_lat, 9 * sizeof(double)},
      {ctx->d_nac, nac * sizeof(double)},
  };
  for (const Arr& a : arrs) {
    const uint64_t n = a.bytes;
    H.add(&n, sizeof(n));
    if (a.p && a.bytes) {
      const elph_status st = hash_device(ctx, a.p, a.bytes, &H, buf);
      if (st != ELPH_OK) return st;
    }
  }
  *out = H.h;
  return ELPH_OK;
}

static SaveHeader make_header(elph_ctx ctx) {
  SaveHeader h;
  std::memset(&h, 0, sizeof(h));
  h.nb = ctx->nb;
  h.na = ctx->na;
  h.nre = ctx->nre;
  h.nrp = ctx->nrp;
  for (int d = 0; d < 3; ++d) h.mesh[d] = ctx->mesh[d];
  h.precision = ctx->precision;
  h.delta = ctx->delta;
  h.frohlich = ctx->frohlich ? 1 : 0;
  h.mu = ctx->mu;
  h.window = ctx->window;
  h.sigma = ctx->sigma;
  h.omega_min = ctx->omega_min;
  h.nk = ctx->nk;
  h.nkept = ctx->nkept;
  h.nstates = ctx->nstates;
  h.store_f32 = ctx->store_f32 ? 1 : 0;
  h.rho_valid = ctx->rho_valid ? 1 : 0;
  h.rho_stride = ctx->rho_stride;
  return h;
}

struct FileCloser {
  void operator()(FILE* f) const {
    if (f) std::fclose(f);
  }
};

// the saved arrays: device pointer and bytes, in file order
struct Part {
  void* d;
  size_t bytes;
  bool table;  // compared on load (tables) or uploaded (store)
};

static std::vector<Part> parts(elph_ctx ctx, bool store_f32, bool rho) {
  const int64_t M = ctx->nstates, nm = ctx->nk * ctx->nbr;
  const size_t nt = (size_t)M * M * ctx->nbr, esz = store_f32 ? 4 : 8;
  std::vector<Part> p = {
      {ctx->d_state_k, (size_t)M * sizeof(int32_t), true},
      {ctx->d_state_m, (size_t)M * sizeof(int32_t), true},
      {ctx->d_eps, (size_t)M * sizeof(double), true},
      {ctx->d_vel, (size_t)M * 3 * sizeof(double), true},
      {ctx->d_hw, (size_t)nm * sizeof(double), true},
      {ctx->d_vph, (size_t)nm * 3 * sizeof(double), true},
      {ctx->d_U, (size_t)ctx->nkept * ctx->nb * ctx->nb * sizeof(cd), true},
      {ctx->d_Bp, nt * esz, false},
      {ctx->d_Bm, nt * esz, false},
  };
  if (rho) p.push_back({ctx->d_rho, (size_t)M * M * ctx->rho_stride, false});
  return p;
}

}  // namespace

elph_status save_state(elph_ctx ctx, const char* path) {
  if (!path || !*path) {
    ctx->err = "null or empty path";
    return ELPH_EINVAL;
  }
  if (!ctx->store_ready) {
    ctx->err = "nothing to save: no vertex store (call elph_scatt_rates or elph_transition_probs with store_B first)";
    return ELPH_ESTATE;
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  SaveHeader h = make_header(ctx);
  elph_status st = input_hash(ctx, &h.input_hash);
  if (st != ELPH_OK) return st;
  std::unique_ptr<FILE, FileCloser> f(std::fopen(path, "wb"));
  if (!f) {
    ctx->err = std::string("cannot open ") + path + " for writing";
    return ELPH_EINVAL;
  }
  Hasher H;
  auto put = [&](const void* p, size_t n) -> bool {
    H.add(p, n);
    return std::fwrite(p, 1, n, f.get()) == n;
  };
  bool ok = put(kMagic, sizeof(kMagic)) && put(&h, sizeof(h));
  std::vector<char> buf(kStage);
  for (const Part& p : parts(ctx, ctx->store_f32, ctx->rho_valid)) {
    for (size_t o = 0; ok && o < p.bytes; o += kStage) {
      const size_t n = std::min(kStage, p.bytes - o);
      HIPCHK(hipMemcpy(buf.data(), (const char*)p.d + o, n, hipMemcpyDeviceToHost));
      ok = put(buf.data(), n);
    }
  }
  const uint64_t sum = H.h;
  ok = ok && std::fwrite(&sum, 1, sizeof(sum), f.get()) == sizeof(sum);
  ok = ok && std::fflush(f.get()) == 0;
  if (!ok) {
    ctx->err = std::string("write to ") + path + " failed";
    return ELPH_EINVAL;
  }
  return ELPH_OK;
}

elph_status load_state(elph_ctx ctx, const char* path) {
  if (!path || !*path) {
    ctx->err = "null or empty path";
    return ELPH_EINVAL;
  }
  std::unique_ptr<FILE, FileCloser> f(std::fopen(path, "rb"));
  if (!f) {
    ctx->err = std::string("cannot open ") + path;
    return ELPH_EINVAL;
  }
  Hasher H;
  auto get = [&](void* p, size_t n) -> bool {
    if (std::fread(p, 1, n, f.get()) != n) return false;
    H.add(p, n);
    return true;
  };
  char magic[8];
  SaveHeader h;
  if (!get(magic, sizeof(magic)) || std::memcmp(magic, kMagic, sizeof(kMagic)) != 0 || !get(&h, sizeof(h))) {
    ctx->err = std::string(path) + " is not a saved context state";
    return ELPH_EINVAL;
  }
  const SaveHeader mine = make_header(ctx);
  if (h.nb != mine.nb || h.na != mine.na || h.nre != mine.nre || h.nrp != mine.nrp || h.mesh[0] != mine.mesh[0] ||
      h.mesh[1] != mine.mesh[1] || h.mesh[2] != mine.mesh[2] || h.precision != mine.precision ||
      h.delta != mine.delta || h.frohlich != mine.frohlich || h.mu != mine.mu || h.window != mine.window ||
      h.sigma != mine.sigma || h.omega_min != mine.omega_min) {
    ctx->err = "saved state belongs to other sizes, parameters, precision form or delta method";
    return ELPH_EINVAL;
  }
  if ((h.store_f32 != 0) != (ctx->precision != ELPH_FP64) || (h.rho_valid && h.rho_stride != (h.na * 3 <= 8 ? 8 : 16))) {
    ctx->err = "saved store layout does not match this context";
    return ELPH_EINVAL;
  }
  uint64_t hash = 0;
  elph_status st = input_hash(ctx, &hash);
  if (st != ELPH_OK) return st;
  if (hash != h.input_hash) {
    ctx->err = "saved state belongs to other inputs (H, D, g, cells, masses or polar terms differ)";
    return ELPH_EINVAL;
  }
  st = build_tables(ctx);
  if (st != ELPH_OK) return st;
  if (h.nk != ctx->nk || h.nkept != ctx->nkept || h.nstates != ctx->nstates) {
    ctx->err = "saved state has another window (kept k or active states differ)";
    return ELPH_EINVAL;
  }
  // store buffers of this context
  const size_t nt = (size_t)ctx->nstates * ctx->nstates * ctx->nbr, esz = h.store_f32 ? 4 : 8;
  ctx->store_ready = false;
  ctx->rates_valid = false;
  ctx->rho_valid = false;
  if (!ctx->d_Bp) {
    void *a = nullptr, *b = nullptr;
    if (dev_alloc(ctx, &a, nt * esz) != hipSuccess || dev_alloc(ctx, &b, nt * esz) != hipSuccess) {
      (void)hipGetLastError();
      dev_free(ctx, a);
      ctx->err = "device allocation of the vertex store failed";
      return ELPH_ENOMEM;
    }
    ctx->d_Bp = a;
    ctx->d_Bm = b;
  }
  if (h.rho_valid) {
    st = refine_prepare(ctx);
    if (st != ELPH_OK) return st;
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  std::vector<char> buf(kStage), dev(kStage);
  for (const Part& p : parts(ctx, h.store_f32 != 0, h.rho_valid != 0)) {
    for (size_t o = 0; o < p.bytes; o += kStage) {
      const size_t n = std::min(kStage, p.bytes - o);
      if (!get(buf.data(), n)) {
        ctx->err = std::string(path) + " is truncated";
        return ELPH_EINVAL;
      }
      if (p.table) {
        HIPCHK(hipMemcpy(dev.data(), (const char*)p.d + o, n, hipMemcpyDeviceToHost));
        if (std::memcmp(dev.data(), buf.data(), n) != 0) {
          ctx->err = "the rebuilt tables differ from the saved ones (another library version or device)";
          return ELPH_EINVAL;
        }
      } else {
        HIPCHK(hipMemcpy((char*)p.d + o, buf.data(), n, hipMemcpyHostToDevice));
      }
    }
  }
  const uint64_t want = H.h;
  uint64_t sum = 0;
  if (std::fread(&sum, 1, sizeof(sum), f.get()) != sizeof(sum) || sum != want) {
    ctx->err = std::string(path) + " is corrupt (checksum mismatch)";
    return ELPH_EINVAL;
  }
  ctx->store_f32 = h.store_f32 != 0;
  ctx->rho_valid = h.rho_valid != 0;
  ctx->store_ready = true;
  return ELPH_OK;
}

}  // namespace elph
