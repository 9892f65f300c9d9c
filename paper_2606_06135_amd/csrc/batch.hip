// Batched SIMPLE iterations of independent contexts (e.g. one geometry at many
// angles of attack, on grids of different sizes) as one HIP graph: the
// iterations of every context are captured once, each context on a capture
// stream of its own (created for the capture and released after it) between a
// fork and a join event of the batch stream, with a fixed
// PCG iteration count and no host read, so one graph launch advances all
// contexts by two SIMPLE iterations with no host synchronisation.  A device
// record per context counts the iterations and keeps the first iteration whose
// maximum normalised residual is <= tol (convergence flag), and flags
// non-finite residuals.
#include "device_common.h"

#include <cmath>
#include <string>
#include <vector>

struct hfdib_batch {
  std::vector<hfdib_ctx*> ctx;
  hipStream_t stream;
  int own_stream;  // created by the batch (no caller stream given)
  hipGraph_t graph;
  hipGraphExec_t exec;
  hipEvent_t fork;
  std::vector<hipEvent_t> join;
  int pcg_iters;
  double tol;
  std::string err;
};

namespace hfdib {

// iterations done, first converged iteration (-1: not yet), non-finite flag
__global__ void k_conv_reset(double* S) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    S[SC_CONV] = 0.0;
    S[SC_CONV + 1] = -1.0;
    S[SC_CONV + 2] = 0.0;
  }
}
__global__ void k_conv_record(double* S, double tol) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double it = S[SC_CONV] + 1.0;
  S[SC_CONV] = it;
  double mx = 0.0;
  bool finite = true;
  for (int q = 0; q < 6; ++q) {
    double r = S[SC_RES + q];
    if (!isfinite(r)) finite = false;
    mx = r > mx ? r : mx;
  }
  if (!finite) S[SC_CONV + 2] = 1.0;
  if (finite && S[SC_CONV + 1] < 0.0 && mx <= tol) S[SC_CONV + 1] = it;
}

static int batch_fail(hfdib_batch* b, const char* what, hipError_t e) {
  b->err = std::string(what) + ": " + hipGetErrorString(e);
  return HFDIB_EDEVICE;
}

}  // namespace hfdib

using namespace hfdib;

extern "C" {

int hfdib_batch_create(hfdib_ctx* const* ctxs, int n, int pcg_iters, double tol, void* hip_stream,
                       hfdib_batch** out) {
  if (!ctxs || n < 1 || pcg_iters < 1 || !out) return HFDIB_EINVAL;
  *out = nullptr;
  hipStream_t bs = (hipStream_t)hip_stream;
  for (int i = 0; i < n; ++i) {
    hfdib_ctx* c = ctxs[i];
    if (!c) return HFDIB_EINVAL;
    if (!c->ready) return HFDIB_ESTATE;
    if (bs && c->stream == bs) return HFDIB_EINVAL;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) return HFDIB_EINVAL;
  }
  hfdib_batch* b = new hfdib_batch();
  b->ctx.assign(ctxs, ctxs + n);
  b->own_stream = 0;
  if (!bs) {
    if (hipStreamCreateWithFlags(&bs, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return HFDIB_EDEVICE;
    }
    b->own_stream = 1;
  }
  b->stream = bs;
  b->graph = nullptr;
  b->exec = nullptr;
  b->pcg_iters = pcg_iters;
  b->tol = tol;
  hipError_t e;
  if ((e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming)) != hipSuccess) {
    if (b->own_stream) (void)hipStreamDestroy(bs);
    delete b;
    return HFDIB_EDEVICE;
  }
  b->join.resize(n);
  for (int i = 0; i < n; ++i)
    if ((e = hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming)) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipEventDestroy(b->join[j]);
      (void)hipEventDestroy(b->fork);
      if (b->own_stream) (void)hipStreamDestroy(bs);
      delete b;
      return HFDIB_EDEVICE;
    }
  // eager set-up outside the capture: the convergence records, everything
  // finished before capturing
  for (hfdib_ctx* c : b->ctx) {
    hipLaunchKernelGGL(k_conv_reset, dim3(1), dim3(64), 0, c->stream, c->scal + SCAL_PCG);
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) {
      int st = batch_fail(b, "batch set-up", e);
      hfdib_batch_destroy(b);
      return st;
    }
  }
  if ((e = hipStreamSynchronize(bs)) != hipSuccess) {
    int st = batch_fail(b, "batch set-up", e);
    hfdib_batch_destroy(b);
    return st;
  }
  // one capture stream per context (default priority), so that every context
  // becomes an independent branch of the graph
  std::vector<hipStream_t> cs(n, nullptr);
  for (int i = 0; i < n; ++i)
    if ((e = hipStreamCreateWithFlags(&cs[i], hipStreamNonBlocking)) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipStreamDestroy(cs[j]);
      int st = batch_fail(b, "capture streams", e);
      hfdib_batch_destroy(b);
      return st;
    }
  // capture two SIMPLE iterations of every context (the pressure buffers swap
  // each iteration, so two leave the host-side pointers as they were)
  if ((e = hipStreamBeginCapture(bs, hipStreamCaptureModeGlobal)) != hipSuccess) {
    for (hipStream_t q : cs) (void)hipStreamDestroy(q);
    int st = batch_fail(b, "begin capture", e);
    hfdib_batch_destroy(b);
    return st;
  }
  int status = HFDIB_OK;
  (void)hipEventRecord(b->fork, bs);
  for (int i = 0; i < n && status == HFDIB_OK; ++i) {
    hfdib_ctx* c = b->ctx[i];
    hipStream_t own = c->stream;
    c->stream = cs[i];
    (void)hipStreamWaitEvent(c->stream, b->fork, 0);
    c->graph_mode = 1;
    c->graph_pcg = pcg_iters;
    for (int it = 0; it < 2 && status == HFDIB_OK; ++it) {
      status = simple_step(c, it, nullptr);
      hipLaunchKernelGGL(k_conv_record, dim3(1), dim3(64), 0, c->stream, c->scal + SCAL_PCG, tol);
    }
    c->graph_mode = 0;
    if (status != HFDIB_OK) b->err = c->err;
    (void)hipEventRecord(b->join[i], c->stream);
    (void)hipStreamWaitEvent(bs, b->join[i], 0);
    c->stream = own;
  }
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(bs, &graph);
  for (hipStream_t q : cs) (void)hipStreamDestroy(q);
  if (status != HFDIB_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    if (status == HFDIB_OK) status = batch_fail(b, "end capture", e);
    hfdib_batch_destroy(b);
    return status;
  }
  b->graph = graph;
  if ((e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
    int st = batch_fail(b, "graph instantiate", e);
    hfdib_batch_destroy(b);
    return st;
  }
  *out = b;
  return HFDIB_OK;
}

int hfdib_batch_run(hfdib_batch* b, int iters) {
  if (!b || iters < 0) return HFDIB_EINVAL;
  hipError_t e;
  // work queued on the contexts' own streams must finish first
  for (hfdib_ctx* c : b->ctx) {
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return batch_fail(b, "batch run", e);
  }
  for (int l = 0; l < (iters + 1) / 2; ++l)
    if ((e = hipGraphLaunch(b->exec, b->stream)) != hipSuccess) return batch_fail(b, "graph launch", e);
  return HFDIB_OK;
}

int hfdib_batch_status(hfdib_batch* b, int* conv_iter, int* iters_done, double* res) {
  if (!b) return HFDIB_EINVAL;
  hipError_t e;
  if ((e = hipStreamSynchronize(b->stream)) != hipSuccess) return batch_fail(b, "batch sync", e);
  int status = HFDIB_OK;
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    hfdib_ctx* c = b->ctx[i];
    double h[9];
    if ((e = hipMemcpy(h, c->scal + SCAL_PCG + SC_CONV, 3 * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)
      return batch_fail(b, "batch status", e);
    if ((e = hipMemcpy(h + 3, c->scal + SCAL_PCG + SC_RES, 6 * sizeof(double), hipMemcpyDeviceToHost)) !=
        hipSuccess)
      return batch_fail(b, "batch status", e);
    if (iters_done) iters_done[i] = (int)h[0];
    if (conv_iter) conv_iter[i] = (int)h[1];
    if (res)
      for (int q = 0; q < 6; ++q) res[6 * i + q] = h[3 + q];
    if (h[2] != 0.0) status = HFDIB_EDIVERGED;
  }
  return status;
}

const char* hfdib_batch_last_error(const hfdib_batch* b) { return b ? b->err.c_str() : "null batch"; }

void hfdib_batch_destroy(hfdib_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (hipEvent_t ev : b->join)
    if (ev) (void)hipEventDestroy(ev);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->own_stream && b->stream) {
    (void)hipStreamSynchronize(b->stream);
    (void)hipStreamDestroy(b->stream);
  }
  delete b;
}

}  // extern "C"
