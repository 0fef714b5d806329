// Host pipeline: frames from host memory through the detector to a CPU
// consumer stage (Sec. V-C, pipelining: the GPU detects faces in one batch
// of frames while CPU threads process the detections of the previous one;
// Sec. V-A, data transfers between host and device).
//
// A pipeline owns `depth` stages.  A stage is a stream with its own device
// frame buffer, workspace, detection buffers and page-locked host buffers.
// submit() takes a free stage, puts the frames on the device (through the
// stage's page-locked staging buffer, or straight from the caller's
// memory), enqueues hog_detect_batch and the copy of the detections back,
// and returns; consumer threads wait for a stage's event, hand its
// detections to the consumer callback and free the stage.  So while the
// GPU works on one batch, the host copies the next batch in and the
// consumers process the last one.
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include <string.h>

#include "hog_internal.h"

namespace {

struct Stage {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint8_t* h_frames = nullptr;   // page-locked staging [batch][h][w]
    uint8_t* d_frames = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    hog_det* d_dets = nullptr;
    int* d_n = nullptr;
    hog_det* h_dets = nullptr;     // page-locked [batch][cap]
    int* h_n = nullptr;            // page-locked [batch]
    int n = 0;
    int64_t first = 0;
    int status = HOG_OK;
};

}  // namespace

struct hog_pipeline {
    hog_params prm{};
    hog_pipeline_config cfg{};
    const float* filters = nullptr;
    const float* bias = nullptr;
    int nf = 0;
    int device = 0;
    std::vector<Stage> stages;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<int> free_stages;   // stages ready for submit()
    std::deque<int> ready;         // submitted stages in submission order
    int in_flight = 0;             // submitted and not yet consumed
    bool stop = false;
    int error = HOG_OK;            // first error of a submit or a batch
    std::vector<std::thread> workers;
};

namespace {

// Frees what create allocated (teardown: errors are not actionable here).
void release(hog_pipeline* p) {
    for (Stage& s : p->stages) {
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        if (s.h_frames) (void)hipHostFree(s.h_frames);
        if (s.h_dets) (void)hipHostFree(s.h_dets);
        if (s.h_n) (void)hipHostFree(s.h_n);
        if (s.d_frames) (void)hipFree(s.d_frames);
        if (s.ws) (void)hipFree(s.ws);
        if (s.d_dets) (void)hipFree(s.d_dets);
        if (s.d_n) (void)hipFree(s.d_n);
    }
    p->stages.clear();
}

void consumer_loop(hog_pipeline* p) {
    // the pipeline's device for this thread's HIP calls (a failure shows up
    // as an error of the event wait below)
    (void)hipSetDevice(p->device);
    for (;;) {
        int idx;
        {
            std::unique_lock<std::mutex> lk(p->mu);
            p->cv.wait(lk, [&] { return p->stop || !p->ready.empty(); });
            if (p->ready.empty()) return;   // stop, nothing left
            idx = p->ready.front();
            p->ready.pop_front();
        }
        Stage& s = p->stages[idx];
        int st = s.status;
        if (st == HOG_OK && hipEventSynchronize(s.done) != hipSuccess) st = HOG_E_HIP;
        if (st == HOG_OK && p->cfg.consumer)
            p->cfg.consumer(p->cfg.user, s.first, s.n, s.h_dets, s.h_n, p->cfg.cap);
        {
            std::lock_guard<std::mutex> lk(p->mu);
            if (st != HOG_OK && p->error == HOG_OK) p->error = st;
            p->free_stages.push_back(idx);
            --p->in_flight;
        }
        p->cv.notify_all();
    }
}

}  // namespace

extern "C" {

int hog_pipeline_create(hog_pipeline** out, const hog_params* prm, const hog_pipeline_config* cfg,
                        const float* filters, const float* bias, int nf) {
    if (!out || !prm || !cfg || !filters || !bias) return HOG_E_INVAL;
    *out = nullptr;
    if (prm->regions) return HOG_E_INVAL;
    if (prm->score_arith != HOG_ARITH_F32 && prm->score_arith != HOG_ARITH_F16X3) return HOG_E_INVAL;
    const hog_pipeline_config& c = *cfg;
    if (c.batch < 1 || c.batch > 1024 || c.depth < 1 || c.depth > 16 || c.cap < 1 || c.cap > HOG_MAX_DETS ||
        c.consumer_threads < 1 || c.consumer_threads > 64 || (c.staging != 0 && c.staging != 1))
        return HOG_E_INVAL;
    const size_t ws_bytes = hog_workspace_bytes(c.h, c.w, prm->upsample, c.batch, nf);
    if (ws_bytes == 0) return HOG_E_INVAL;
    hog_pipeline* p = new hog_pipeline();
    p->prm = *prm;
    p->cfg = c;
    p->filters = filters;
    p->bias = bias;
    p->nf = nf;
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return HOG_E_HIP;
    }
    const size_t fbytes = (size_t)c.batch * c.h * c.w;
    p->stages.resize(c.depth);
    bool ok = true;
    for (Stage& s : p->stages) {
        s.ws_bytes = ws_bytes;
        ok = ok && hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&s.done, hipEventDisableTiming) == hipSuccess;
        ok = ok && hipHostMalloc((void**)&s.h_frames, fbytes, hipHostMallocDefault) == hipSuccess;
        ok = ok && hipHostMalloc((void**)&s.h_dets, sizeof(hog_det) * c.batch * c.cap, hipHostMallocDefault) ==
                       hipSuccess;
        ok = ok && hipHostMalloc((void**)&s.h_n, sizeof(int) * c.batch, hipHostMallocDefault) == hipSuccess;
        ok = ok && hipMalloc((void**)&s.d_frames, fbytes) == hipSuccess;
        ok = ok && hipMalloc(&s.ws, ws_bytes) == hipSuccess;
        ok = ok && hipMalloc((void**)&s.d_dets, sizeof(hog_det) * c.batch * c.cap) == hipSuccess;
        ok = ok && hipMalloc((void**)&s.d_n, sizeof(int) * c.batch) == hipSuccess;
        if (!ok) break;
    }
    if (!ok) {
        release(p);
        delete p;
        return HOG_E_HIP;
    }
    for (int i = 0; i < c.depth; ++i) p->free_stages.push_back(i);
    for (int i = 0; i < c.consumer_threads; ++i) p->workers.emplace_back(consumer_loop, p);
    *out = p;
    return HOG_OK;
}

int hog_pipeline_submit(hog_pipeline* p, const uint8_t* frames, int n, int64_t first_frame) {
    if (!p || !frames || n < 1 || n > p->cfg.batch) return HOG_E_INVAL;
    int idx;
    {
        std::unique_lock<std::mutex> lk(p->mu);
        p->cv.wait(lk, [&] { return !p->free_stages.empty(); });
        idx = p->free_stages.front();
        p->free_stages.pop_front();
        ++p->in_flight;
    }
    Stage& s = p->stages[idx];
    const hog_pipeline_config& c = p->cfg;
    const size_t bytes = (size_t)n * c.h * c.w;
    s.n = n;
    s.first = first_frame;
    s.status = HOG_OK;
    const uint8_t* src = frames;
    if (c.staging) {
        memcpy(s.h_frames, frames, bytes);
        src = s.h_frames;
    }
    if (hipMemcpyAsync(s.d_frames, src, bytes, hipMemcpyHostToDevice, s.stream) != hipSuccess) s.status = HOG_E_HIP;
    if (s.status == HOG_OK)
        s.status = hog_detect_batch(&p->prm, s.d_frames, n, c.h, c.w, c.w, (int64_t)c.h * c.w, p->filters, p->bias,
                                    p->nf, s.d_dets, c.cap, s.d_n, s.ws, s.ws_bytes, s.stream);
    if (s.status == HOG_OK &&
        (hipMemcpyAsync(s.h_dets, s.d_dets, sizeof(hog_det) * n * c.cap, hipMemcpyDeviceToHost, s.stream) !=
             hipSuccess ||
         hipMemcpyAsync(s.h_n, s.d_n, sizeof(int) * n, hipMemcpyDeviceToHost, s.stream) != hipSuccess ||
         hipEventRecord(s.done, s.stream) != hipSuccess))
        s.status = HOG_E_HIP;
    const int st = s.status;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        p->ready.push_back(idx);
    }
    p->cv.notify_all();
    return st;
}

int hog_pipeline_drain(hog_pipeline* p) {
    if (!p) return HOG_E_INVAL;
    std::unique_lock<std::mutex> lk(p->mu);
    p->cv.wait(lk, [&] { return p->in_flight == 0; });
    const int e = p->error;
    p->error = HOG_OK;
    return e;
}

int hog_pipeline_destroy(hog_pipeline* p) {
    if (!p) return HOG_E_INVAL;
    const int e = hog_pipeline_drain(p);
    {
        std::lock_guard<std::mutex> lk(p->mu);
        p->stop = true;
    }
    p->cv.notify_all();
    for (std::thread& t : p->workers) t.join();
    release(p);
    delete p;
    return e;
}

}  // extern "C"
