// Internal plumbing of libsfmm: error handling, the device memory pool,
// device vectors, and the launch wrappers that the host driver calls.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace sfmm {

// A failure anywhere below the C ABI is thrown as one of these and turned
// into a status code + message at the boundary.
struct Error : std::runtime_error {
    int status;
    Error(int s, const std::string& m) : std::runtime_error(m), status(s) {}
};

enum { ST_OK = 0, ST_INVALID_ARG = 1, ST_OOM = 2, ST_HIP = 3, ST_TOL = 4, ST_INTERNAL = 5 };

#define SFMM_HIP(call)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::sfmm::Error(::sfmm::ST_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

#define SFMM_LAUNCH_CHECK() SFMM_HIP(hipGetLastError())

// Caching device allocator: freed blocks are kept per size class and reused,
// so steady-state planning does no hipMalloc.
void* pool_alloc(size_t bytes);
void pool_free(void* p);
void pool_release_all();

template <typename T>
struct DVec {
    T* p = nullptr;
    size_t n = 0, cap = 0;
    DVec() = default;
    DVec(const DVec&) = delete;
    DVec& operator=(const DVec&) = delete;
    ~DVec() { reset(); }
    void reset() {
        if (p) pool_free(p);
        p = nullptr;
        n = cap = 0;
    }
    // resize without keeping contents
    void resize(size_t m) {
        if (m > cap) {
            reset();
            cap = m + m / 4 + 64;
            p = (T*)pool_alloc(cap * sizeof(T));
        }
        n = m;
    }
    // grow keeping contents (stream-ordered copy)
    void grow(size_t m, hipStream_t s) {
        if (m > cap) {
            size_t c2 = m + m / 2 + 64;
            T* q = (T*)pool_alloc(c2 * sizeof(T));
            if (p && n) SFMM_HIP(hipMemcpyAsync(q, p, n * sizeof(T), hipMemcpyDeviceToDevice, s));
            if (p) {
                // the pool may hand this block out again: make the copy finish first
                SFMM_HIP(hipStreamSynchronize(s));
                pool_free(p);
            }
            p = q;
            cap = c2;
        }
        n = m;
    }
    T* data() const { return p; }
    size_t size() const { return n; }
};

constexpr int kMaxOrder = 48;

// ---------------------------------------------------------------- utilities
void fill_f64(double* p, size_t n, double v, hipStream_t s);
void fill_i32(int* p, size_t n, int v, hipStream_t s);
// exclusive scan of n ints; the total goes to *total (device)
void scan_excl_i32(const int* in, int* out, int64_t n, int* total, hipStream_t s);
// stable LSD radix sort of (key, value) pairs on key bits [begin_bit, bits)
void radix_sort_u64(uint64_t* keys, uint32_t* vals, int64_t n, int bits, hipStream_t s, int begin_bit = 0);
void sum_f64(const double* x, int64_t n, double* out, hipStream_t s);
void sum_i64(const long long* x, int64_t n, long long* out, hipStream_t s);

// ---------------------------------------------------------------- tree
// Copy [3][n] planes, check they are unit vectors (err bit 1: non-finite,
// bit 2: off the sphere by more than 1e-6), renormalise ones off by more
// than 1e-14, and compute their order-29 keys.
void prepare_points(const double* in, int64_t n, double* x, double* y, double* z, uint64_t* keys,
                    uint32_t* idx, int* err, hipStream_t s);
void gather_points(const uint32_t* idx, int64_t n, const double* x, const double* y, const double* z,
                   const double* q_in, double* ox, double* oy, double* oz, double* oq, hipStream_t s);
void tree_base_level(const uint64_t* keys, int64_t n, int* level, uint64_t* pixel, int* first, int* count,
                     int* parent, int* child0, hipStream_t s);
void tree_split_flags(int b0, int nb, const int* level, const int* count, int m, int max_level, int* flag,
                      hipStream_t s);
void tree_make_children(int b0, int nb, int child_base, const int* flag, const int* off, const uint64_t* keys,
                        int* level, uint64_t* pixel, int* first, int* count, int* parent, int* child0,
                        hipStream_t s);
void box_geometry(int nb, const int* level, const uint64_t* pixel, double* cen /*[nb][4]: x,y,z,rho*/,
                  double* rad, double* gdd /*[nb][8]*/, hipStream_t s);
void locate_targets(const uint64_t* keys, int64_t m, const int* child0, const int* level, int* leaf,
                    hipStream_t s);
void target_ranges(const int* leaf, int64_t m, int* tfirst, int* tcount, hipStream_t s);
void flag_nonzero(const int* count, int n, int* flag, hipStream_t s);
void compact_index(const int* flag, const int* off, int n, int* out, hipStream_t s);

// walk
struct WalkCtx {
    const int* child0;
    const int* count;
    const double* cen;
    const double* rad;
    const double* gdd;
    double c_s, c_t;
};
void walk_classify(const int2* F, int n, const WalkCtx& w, uint8_t* action, int* nchild, int* nm2l, int* np2p,
                   hipStream_t s);
void walk_emit(const int2* F, int n, const WalkCtx& w, const uint8_t* action, const int* ochild,
               const int* om2l, const int* op2p, int2* Fnext, uint64_t* m2l, int m2l_base, uint64_t* p2p,
               int p2p_base, hipStream_t s);
void m2l_order_keys(const int* off, int nbox, uint64_t* keys, uint32_t* vals, hipStream_t s);
// pairs (target << 32 | source) sorted by target -> CSR offsets and sources
void pairs_to_csr(const uint64_t* sorted, int npairs, int nbox, int* off /*[nbox+1]*/, int* src, hipStream_t s);
// sort keys putting the target leaves with the most direct-act work first
// (targets x close leaves); flag the leaves that have any
void work_order_keys(const int* off, const int* tcount, int n, uint64_t* keys, uint32_t* vals, int* flag,
                     hipStream_t s);
// particle-target pairs of each leaf's direct acts: tcount[T] * sum count[S]
// ---------------------------------------------------------------- fmm
struct FmmCtx {
    int p;
    const double* cen;   // [nb][4] x, y, z, rho
    const double* rad;   // [nb] box radius R
    const int* level;
    const int* first;
    const int* count;
    const int* parent;
    const int* child0;
    const double* sx;
    const double* sy;
    const double* sz;
    const double* sq;
    double* mult;        // [nb][2p+2]
    double* local;       // [nb][2p+2]
};
void fmm_p2m(const FmmCtx& c, int nb, hipStream_t s);
void fmm_m2m(const FmmCtx& c, int b0, int nb, hipStream_t s);
void fmm_m2l(const FmmCtx& c, const int* order, int n, const int* off, const int* src, hipStream_t s);
void fmm_l2l(const FmmCtx& c, int b0, int nb, hipStream_t s);
void fmm_l2p(const FmmCtx& c, const double* tx, const double* ty, const double* tz, const int* tleaf,
             const uint32_t* tperm, int64_t m, double psi_shift, double* psi, double* defl, int64_t m_out,
             hipStream_t s);
void fmm_p2p(const FmmCtx& c, const int* tleaves, int ntl, const int* off, const int* src, const int* tfirst,
             const int* tcount, const double* tx, const double* ty, const double* tz, const uint32_t* tperm,
             double* psi, double* defl, int64_t m_out, hipStream_t s);
void near_work(const FmmCtx& c, const int* tleaves, int ntl, const int* off, const int* src, const int* tfirst,
               const int* tcount, const double* tx, const double* ty, const double* tz, long long* pairs,
               long long* evals, hipStream_t s);
void fmm_m2p(const FmmCtx& c, const int* tleaves, int ntl, const int* off, const int* src, const int* tfirst,
             const int* tcount, const double* tx, const double* ty, const double* tz, const uint32_t* tperm,
             double* psi, double* defl, int64_t m_out, hipStream_t s);

}  // namespace sfmm
