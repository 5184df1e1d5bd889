// gpa_attribute_noalloc: the sample histogram and the instruction blamer of
// one profile into caller-given device arrays, with the histogram's scratch
// taken from a fixed device array of this file instead of the allocator.
//
// The array is a file-scope __device__ symbol, so every GPU the library runs
// on holds its own copy from the module's load until the process ends.  Its
// address on a device is looked up once, with that device current, and kept;
// the kernels receive that address (the symbol's name in host code is only a
// host-side stand-in).
#include <map>
#include <mutex>

#include "common.h"

namespace gpa {
namespace {

constexpr size_t kScratchBytes = (size_t)192 << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;   // device -> address of its copy of scratch

// the current device's copy of scratch
void *scratch_on_current_device() {
  int dev = 0;
  GPA_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    set_error("hipGetSymbolAddress of the scratch array failed on device %d: %s", dev,
              hipGetErrorString(e));
    throw Error{GPA_E_DEVICE};
  }
  g_scratch_ptr[dev] = ptr;
  return ptr;
}

}  // namespace
}  // namespace gpa

using namespace gpa;

extern "C" {

uint64_t gpa_noalloc_scratch_bytes(void) { return kScratchBytes; }

gpa_status gpa_attribute_noalloc(const gpa_program *p, const gpa_sample *samples, uint64_t n,
                                 void *stream, uint32_t *counts, uint64_t *totals, double *share,
                                 double *blamed, double *self_, double *fine) {
  if (!p || (n && !samples) || !counts || !totals || !blamed || !self_ || !fine ||
      (!share && p->n_edges * p->n_blamable > 0)) {
    set_error("gpa_attribute_noalloc: NULL argument");
    return GPA_E_INVALID;
  }
  if (n >= 0x40000000ull) {
    set_error("gpa_attribute_noalloc: 2^30 samples or more");
    return GPA_E_UNSUPPORTED;
  }
  if (p->n_instr > hist_hot_max_pcs()) {
    set_error("gpa_attribute_noalloc: programs of up to %u instructions are supported (this one "
              "has %u)", hist_hot_max_pcs(), p->n_instr);
    return GPA_E_UNSUPPORTED;
  }
  // the issued samples, the histogram's scratch, then the blamer's compact
  // tables (expanded into the caller's full tables at the end), each piece
  // 256-byte aligned
  auto blk = [](size_t bytes) { return (bytes + 255) / 256 * 256; };
  const size_t ni = p->n_instr;
  const size_t need = blk(ni * 4) + hist_hot_scratch_bytes(p->n_instr, n) +
                      blk(ni * p->n_blamable * 2 * 8) + blk(ni * kBlameFx * 8) + blk(ni * 2) + 256;
  if (need > kScratchBytes) {
    set_error("gpa_attribute_noalloc: %llu records of a %u-instruction program need %zu bytes of "
              "scratch, more than the fixed %zu", (unsigned long long)n, p->n_instr, need,
              kScratchBytes);
    return GPA_E_UNSUPPORTED;
  }
  hipStream_t s = (hipStream_t)stream;
  try {
    Arena ar(scratch_on_current_device(), kScratchBytes);
    uint32_t *issued = ar.get<uint32_t>(ni);
    run_hist(*p, samples, n, counts, issued, reinterpret_cast<unsigned long long *>(totals), s, ar,
             /*allow_partition=*/false);
    double *bl = ar.get<double>(ni * p->n_blamable * 2);
    double *fx = ar.get<double>(ni * kBlameFx);
    uint16_t *nocand = ar.get<uint16_t>(ni);
    launch_blame(*p, counts, issued, share, nullptr, bl, fx, nocand, s);
    expand_blame_tables(*p, counts, bl, fx, nocand, blamed, self_, fine, s);
  } catch (const Error &e) {
    return e.code;
  } catch (...) {
    set_error("gpa_attribute_noalloc: unexpected failure");
    return GPA_E_DEVICE;
  }
  return GPA_OK;
}

}  // extern "C"
