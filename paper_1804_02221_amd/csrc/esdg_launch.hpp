// Launch wrappers: one translation unit per polynomial degree instantiates
// Launch<N, double> and Launch<N, float>; the runtime dispatches on N.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace esdg {

template <typename R> struct Tab;
template <typename R> struct Phys;

// Device buffers of one context (typed views are cast per precision).
struct Bufs {
    int N = 0;
    int64_t K = 0;
    double *x = nullptr, *y = nullptr;      // float64 coordinates
    double *xr = nullptr, *yr = nullptr;    // the same less each element's first node (float64 contexts)
    void *Ax = nullptr, *Cx = nullptr, *Ae = nullptr, *Ce = nullptr;
    void *mref = nullptr;                   // float32 contexts: [K][4] metric terms of each element's middle node
    void *bx = nullptr, *by = nullptr, *bface = nullptr, *b = nullptr;
    int32_t *nbr = nullptr;
    int8_t *code = nullptr;
    int walls = 0;           // some side of the mesh is a solid wall
    void *W[3][3] = {};      // state buffers [buffer][h, hu, hv]: W^n and the two stage outputs
    void *dU[3] = {};        // LSRK register
    void *Rb[3] = {};        // right-hand side output scratch
    void *gmax = nullptr;    // [K] max |grad xi|^2 + |grad eta|^2 per element (mesh constant)
    void *tabg = nullptr;    // Tab<R> in device memory
    void *fgeo = nullptr;    // [K][4][nf][3] face unit normals and w_0 J / J^surf (mesh constant)
    void *frec = nullptr;    // [K][4][nf][3] face records (h, u, v) of the state whose bounds are in dtc
    void *dtc = nullptr, *dtv = nullptr;  // [K] per-element CFL / viscous bounds of one state
    void *eps[3] = {};       // [K] element viscosity of each state buffer
    int32_t *list[3] = {};   // [K] elements of each state buffer with eps > 0
    int *count = nullptr;    // [3] list lengths
    void *vtr = nullptr;     // [K][4][nf][4] viscous face fluxes (elements with eps > 0)
    void *lv[2] = {};        // [K][np] viscous terms L^v (momentum rows)
    double *dscal = nullptr; // per instance k: [8k..8k+3] dt and its bounds, [8k+4] time, [8k+5..7] spare
    unsigned long long *slots = nullptr;  // [instance][3][kDtSlots]
    int n_inst = 1;          // instances (ensembles); > 1: the arrays below are set
    int32_t *inst = nullptr;    // [K] instance of each internal element
    int64_t *cstart = nullptr;  // [nchunks + 1] element chunks of the time-step pass (never across instances)
    int32_t *cinst = nullptr;   // [nchunks] instance of each chunk
    int64_t nchunks = 0;
    int *flags = nullptr;    // status flags (kFlag* in esdg_kernels.hpp)
    int *iflags = nullptr;   // [n_inst] per-instance step flags (ensembles): 1 negative mean, 2 step above its result's bounds
    int *imask = nullptr;    // [n_inst] instances whose step is redone at half the size (ensembles)
    double *part = nullptr;  // diagnostics partial sums
    int64_t part_cap = 0;
};

// Optional events recorded by the launch itself around one kernel (timing).
struct Ev {
    hipEvent_t a = nullptr, b = nullptr;
};

struct StageCall {
    int mode;          // kModeRhs, kModeLsrk, kModeSsp
    bool av;           // add the viscous terms of visc()
    int in, out, base; // state buffers: input, output, W^n (SSP)
    bool out_rhs;      // write into Rb instead of W[out]
    double ca, cb;     // stage coefficients
    bool dt_next;      // last stage of a step: leave the output's dt bounds in dtc/dtv
    bool store_du;     // LSRK: write the register dU (not needed after the last stage)
    int variant;       // stage-kernel workgroup size: 0 default, 1 alternative
    bool masked = false;  // ensembles: only the elements of instances with imask set
};

// One reverse stage of the discrete adjoint (float64 contexts only).
struct AdjCall {
    const void *W[3];          // stage input state W_{k-1}
    const void *a[3], *c[3];   // dL/dW_k and A_{k+1} dL/dd_{k+1} (nullptr: zero)
    void *ao[3], *co[3];       // dL/dW_{k-1} and A_k dL/dd_k (co nullptr: not written)
    const void *x[3], *y[3];   // added to ao and to co (nullptr: zero; y may alias co)
    double *gbx, *gby, *gbn;   // bathymetry cotangents, accumulated
    double ca, cb, dt;         // A_k, B_k and the step
    double sa = 1.0;           // scale of a in ao (SSPRK: beta_k)
};

template <int N, typename R>
struct Launch {
    static hipError_t geometry(const Bufs &B, const Tab<double> &td, hipStream_t s);
    static hipError_t bathymetry(const Bufs &B, const double *b, const Tab<double> &td, hipStream_t s);
    static hipError_t indicator(const Bufs &B, int buf, const Phys<R> &P, const Tab<R> &t, hipStream_t s,
                                Ev ev);
    static hipError_t av_faces(const Bufs &B, int in, const Phys<R> &P, const Tab<R> &t, hipStream_t s, Ev ev);
    static hipError_t av_div(const Bufs &B, int in, int reset, const Phys<R> &P, const Tab<R> &t,
                             hipStream_t s, Ev ev);
    static hipError_t stage(const Bufs &B, const StageCall &c, const Phys<R> &P, const Tab<R> &t,
                            hipStream_t s, Ev ev);
    static hipError_t limit(const Bufs &B, int buf, const Phys<R> &P, const Tab<R> &t, hipStream_t s);
    static hipError_t dt(const Bufs &B, int in, bool av, bool fused, const Phys<R> &P, hipStream_t s, Ev ev);
    static hipError_t adjoint_stage(const Bufs &B, const AdjCall &c, const Phys<R> &P, const Tab<R> &t,
                                    hipStream_t s, Ev ev);
    static hipError_t bathymetry_adjoint(const Bufs &B, const Tab<double> &td, const double *gbx,
                                         const double *gby, const double *gbn, double *gb, hipStream_t s);
    static hipError_t diag(const Bufs &B, int buf, const Phys<R> &P, const Tab<R> &t, int64_t *nblocks,
                           hipStream_t s);
    static int threads();
    static int elems_per_block();
};

}  // namespace esdg
