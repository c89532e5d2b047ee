// bie_apply_bio_noalloc: the operator application of bie_apply_bio with its per-call work
// buffers (far-field source strengths, transform coefficients, near-series tables, sphere
// moments, far-field partial sums) in one file-scope device array instead of the
// context's own buffers, for callers that cannot allocate device memory.
#include <map>
#include <mutex>

#include "bie_internal.h"

namespace bie {
namespace {

constexpr size_t kScratchBytes = (size_t)96 << 20;  // BIE_NOALLOC_SCRATCH_BYTES
static_assert(kScratchBytes == BIE_NOALLOC_SCRATCH_BYTES, "header and library disagree on the scratch size");

// Each device holds its own copy of this array for the life of the process.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mtx;
std::map<int, unsigned char*> g_ptr;  // device ordinal -> address of that device's copy

// Address of the current device's copy (the array's name is only a host-side stand-in).
unsigned char* scratch_on(int device) {
  std::lock_guard<std::mutex> lk(g_mtx);
  auto it = g_ptr.find(device);
  if (it != g_ptr.end()) return it->second;
  void* p = nullptr;
  BIE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw Error{BIE_EDEVICE, "hipGetSymbolAddress returned NULL for the scratch array"};
  g_ptr[device] = static_cast<unsigned char*>(p);
  return static_cast<unsigned char*>(p);
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Points the context's work buffers at the scratch array for the lifetime of the guard.
struct ScratchSwap {
  bie_ctx* c;
  void *q, *coef, *neartab, *moments, *partial;
  int nsplit;
  ScratchSwap(bie_ctx* cc, unsigned char* base, size_t oq, size_t oc, size_t ot, size_t om, size_t op, int ns)
      : c(cc), q(cc->q.ptr), coef(cc->coef.ptr), neartab(cc->neartab.ptr), moments(cc->moments.ptr),
        partial(cc->partial.ptr), nsplit(cc->nsplit) {
    c->q.ptr = base + oq;
    c->coef.ptr = base + oc;
    c->neartab.ptr = neartab ? base + ot : nullptr;
    c->moments.ptr = base + om;
    c->partial.ptr = base + op;
    c->nsplit = ns;
  }
  ~ScratchSwap() {
    c->q.ptr = q;
    c->coef.ptr = coef;
    c->neartab.ptr = neartab;
    c->moments.ptr = moments;
    c->partial.ptr = partial;
    c->nsplit = nsplit;
  }
};

void apply_noalloc(bie_ctx* c, int op, int precision, const double* mu, double* u) {
  const int base = op & 0xff;
  if (base != BIE_OP_S && base != BIE_OP_D && base != BIE_OP_SD_BIE && base != BIE_OP_DN_BIE &&
      base != BIE_OP_MOBILITY)
    throw Error{BIE_EINVAL, "bie_apply_bio_noalloc: op must be BIE_OP_S, _D, _SD_BIE, _DN_BIE or _MOBILITY"};
  if ((op & ~(0xff | BIE_STAGE_SELF | BIE_STAGE_NEAR | BIE_STAGE_FAR)) != 0)
    throw Error{BIE_EINVAL, "bie_apply_bio_noalloc: unknown stage bits"};
  if (c->near_method != 0) throw Error{BIE_EINVAL, "bie_apply_bio_noalloc: near_method must be 0"};
  if (precision != BIE_FP64 && precision != BIE_MIXED) throw Error{BIE_EINVAL, "bad precision"};
  // layout: q | coef | near tables | moments | far partial sums (nsplit x N x 3)
  const size_t oq = 0;
  const size_t oc = align256(oq + (size_t)c->N * 4 * sizeof(double));
  const size_t ot = align256(oc + (size_t)c->nb * 3 * c->ncoef * 2 * sizeof(double));
  const size_t om = align256(ot + (c->neartab.ptr ? (size_t)c->nb * c->near_slots * 16 * sizeof(double) : 0));
  const size_t op0 = align256(om + (size_t)c->nb * 6 * sizeof(double));
  const size_t per_split = (size_t)c->N * 3 * sizeof(double);
  if (op0 + per_split > kScratchBytes)
    throw Error{BIE_EINVAL, "bie_apply_bio_noalloc: the work buffers of " + std::to_string(c->nb) + " spheres (" +
                                std::to_string(op0 + per_split) + " bytes) exceed the scratch array (" +
                                std::to_string(kScratchBytes) + " bytes)"};
  const int ns = (int)std::max<size_t>(1, std::min<size_t>((size_t)c->nsplit, (kScratchBytes - op0) / per_split));
  BIE_HIP(hipSetDevice(c->device));
  unsigned char* sbase = scratch_on(c->device);
  ScratchSwap sw(c, sbase, oq, oc, ot, om, op0, ns);
  apply(c, op, precision, mu, u);
}

}  // namespace
}  // namespace bie

extern "C" int bie_apply_bio_noalloc(bie_ctx* c, int op, int precision, const double* mu, double* u) {
  if (!c || !mu || !u) {
    bie::set_error("null argument");
    return BIE_EINVAL;
  }
  if (mu == u) {
    bie::set_error("mu and u alias");
    return BIE_EINVAL;
  }
  try {
    bie::clear_error();
    bie::apply_noalloc(c, op, precision, mu, u);
  } catch (const bie::Error& e) {
    bie::set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    bie::set_error(e.what());
    return BIE_EINVAL;
  }
  return BIE_OK;
}
