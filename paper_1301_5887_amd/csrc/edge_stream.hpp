// Chunked pass over an edge list held in host memory: chunk j is copied into
// one of two buffer pairs on two copy streams of the device while the
// caller's stream runs the consumer on chunk j - 1.  The destination array
// goes by the copy engine; the source array, when it is pinned, by a copy
// kernel that reads it over the host link, so both share the link (pinned
// memory also lets the copies overlap the kernels).
#pragma once

#include "common.hpp"

namespace wedge {

constexpr uint64_t kEdgeChunk = 1ULL << 24;

// Two copy streams per device (which = 0, 1), created on first use (default
// priority) and kept until the process ends.
int copy_stream(hipStream_t* out, int which);

// The device address of host memory [h, h + bytes) when kernels may read it
// directly: pinned memory (hipHostMalloc, torch's pin_memory) whose one
// allocation holds the whole range.  Null for anything else (pageable memory
// goes through hipMemcpyAsync instead).
const char* host_direct(const void* h, size_t bytes);

// Enqueues on cs the copy of n words from host memory read directly (an
// address from host_direct) into b: a kernel that reads over the host link.
int copy_words_direct(const uint32_t* s, uint32_t* b, uint64_t n, hipStream_t cs);

// The events of one pass; destroyed with the pass, on every return path
// (an event may be destroyed while work that records it is pending).
struct EdgeStreamEvents {
  hipEvent_t e[7] = {};  // start, copied[2] (src), copied[2] (dst), used[2]
  ~EdgeStreamEvents() {
    for (hipEvent_t x : e)
      if (x) (void)hipEventDestroy(x);
  }
};

// consume(src, dst, ne) enqueues the work on chunk (src, dst) of ne edges on
// st; buf[b][0] and buf[b][1] hold chunk uint32 each.  Returns the first
// error of a copy, an event call or the consumer.
template <class Consume>
int stream_edges(const uint32_t* h_src, const uint32_t* h_dst, uint64_t m_in, uint64_t chunk,
                 uint32_t* buf[2][2], hipStream_t st, Consume consume) {
  if (m_in == 0) return WEDGE_OK;
  hipStream_t cs, cs2;
  int rc = copy_stream(&cs, 0);
  if (rc) return rc;
  if ((rc = copy_stream(&cs2, 1))) return rc;
  const char* ds = host_direct(h_src, (size_t)m_in * 4);
  EdgeStreamEvents ev;
  for (hipEvent_t& x : ev.e) WEDGE_HIP_TRY(hipEventCreateWithFlags(&x, hipEventDisableTiming));
  hipEvent_t start = ev.e[0];
  const hipEvent_t copied[2] = {ev.e[1], ev.e[2]}, copied2[2] = {ev.e[3], ev.e[4]},
                   used[2] = {ev.e[5], ev.e[6]};
  // the copies may only overwrite the buffers once earlier work on the
  // caller's stream is done with them
  WEDGE_HIP_TRY(hipEventRecord(start, st));
  WEDGE_HIP_TRY(hipStreamWaitEvent(cs, start, 0));
  WEDGE_HIP_TRY(hipStreamWaitEvent(cs2, start, 0));
  const uint64_t nchunks = (m_in + chunk - 1) / chunk;
  for (uint64_t j = 0; j < nchunks && rc == WEDGE_OK; ++j) {
    const int b = (int)(j & 1);
    const uint64_t e0 = j * chunk;
    const uint64_t ne = (m_in - e0) < chunk ? (m_in - e0) : chunk;
    if (j >= 2) {
      WEDGE_HIP_TRY(hipStreamWaitEvent(cs, used[b], 0));
      WEDGE_HIP_TRY(hipStreamWaitEvent(cs2, used[b], 0));
    }
    // src on the first copy stream (by the copy kernel when the memory allows
    // it), dst by the copy engine on the second: both share the host link
    if (ds) {
      rc = copy_words_direct((const uint32_t*)ds + e0, buf[b][0], ne, cs);
      if (rc) return rc;
    } else {
      WEDGE_HIP_TRY(hipMemcpyAsync(buf[b][0], h_src + e0, ne * 4, hipMemcpyHostToDevice, cs));
    }
    WEDGE_HIP_TRY(hipMemcpyAsync(buf[b][1], h_dst + e0, ne * 4, hipMemcpyHostToDevice, cs2));
    WEDGE_HIP_TRY(hipEventRecord(copied[b], cs));
    WEDGE_HIP_TRY(hipEventRecord(copied2[b], cs2));
    WEDGE_HIP_TRY(hipStreamWaitEvent(st, copied[b], 0));
    WEDGE_HIP_TRY(hipStreamWaitEvent(st, copied2[b], 0));
    rc = consume((const uint32_t*)buf[b][0], (const uint32_t*)buf[b][1], ne);
    WEDGE_HIP_TRY(hipEventRecord(used[b], st));
  }
  return rc;
}

}  // namespace wedge
