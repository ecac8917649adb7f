// Internal state of a vsie_handle and host-side setup helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/vsie.h"
#include "vsie_math.h"

namespace vsie {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define VSIE_HIP(call)                                                                     \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      throw ::vsie::Error(VSIE_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
  } while (0)

// RWG functions of one domain (all meshes of that domain concatenated, input order).
struct Rwg {
  std::vector<double> verts;   // 3 * nv
  std::vector<int> tris;       // 3 * nt
  std::vector<double> area;    // nt
  std::vector<int> ea, eb;     // edge vertices, a < b
  std::vector<int> tp, tm;     // T+, T-
  std::vector<int> fp, fm;     // free vertices
  std::vector<int> flp, flm;   // local index of the free vertex in T+ / T-
  std::vector<double> len;
  int m = 0;
  V3 vert(int i) const { return {verts[3 * i], verts[3 * i + 1], verts[3 * i + 2]}; }
};

// Flattened description of an RWG set for device kernels.
struct RwgDev {
  const double* verts;   // 3 nv
  const int* tris;       // 3 nt
  const double* area;    // nt
  const int* tpm;        // [m][2] T+, T-
  const int* flpm;       // [m][2] local index (0..2) of the free vertex inside T+ / T-
  const int* fpm;        // [m][2] free vertex ids
  const double* len;     // m
  int m;
};

struct PortEdge {
  int domain;   // VSIE_NEAR / VSIE_FAR
  int idx;      // RWG index within the domain
  double sign;
};

template <typename R> struct OpData {
  // volume convolution
  cx<R>* spec = nullptr;       // [6][P3/2+1][P2/2+1][P1/2+1], scaled by h^3 / (P1 P2 P3)
  cx<R>* dv_chi = nullptr;     // [n_v] h^3 / chi (0 in air)
  cx<R>* tw[4] = {nullptr, nullptr, nullptr, nullptr};   // twiddles for P1, P2, P3 (index by axis)
  // pFFT
  R* W = nullptr;              // [m_n][3][125]
  R* roww = nullptr;           // [nnz_grid][3]
  cx<R>* projv = nullptr;      // [n_gridrows][3]: projected near currents per projection voxel
  cx<R>* pc_val = nullptr;     // precorrection values
  // ACA
  cx<R>* U = nullptr;          // [m_n][k]
  cx<R>* V = nullptr;          // [m_f][k]
  // TT cores per component: G1 [n1][r1], G2 [r1][n2][r2], G3 [r2][n3][r3], G4 [r3][m_f]
  cx<R>* G[3][4] = {};
  // dense far block
  cx<R>* Zff = nullptr;        // upper-triangle tiles of the symmetric far block
  cx<R>* sym_part = nullptr;   // per-tile partial sums
  cx<R>* multi_part = nullptr; // per-tile partial sums of up to 16 right-hand sides
  // work buffers
  cx<R>* gridA = nullptr;      // [3][ne3][ne2][ne1] (also the convolution output)
  cx<R>* bufB = nullptr;       // [3][ne3][ne2][P1]
  cx<R>* bufC = nullptr;       // [3][ne3][P2][P1]
  cx<R>* tt_work = nullptr;    // TT intermediates
  cx<R>* small_work = nullptr; // ACA / reductions
  cx<R>* dual_part = nullptr;  // partial sums of the one-pass product with V
};

constexpr int LU_NB = 64;   // panel width of the dense LU

// Factors of P A = L U, in place in A (row-major, leading dimension lda). The caller provides the
// device buffers: d_ipiv and d_perm (n ints each), d_info (1 int), Linv and Uinv
// (ceil(n / LU_NB) blocks of LU_NB x LU_NB): the inverted unit-lower and upper diagonal blocks.
struct DenseLU {
  int n = 0;
  int64_t lda = 0;
  cxd* A = nullptr;
  cxd* Linv = nullptr;
  cxd* Uinv = nullptr;
  int* d_ipiv = nullptr;
  int* d_perm = nullptr;
  int* d_info = nullptr;
  std::vector<int> perm;   // row i of L U is row perm[i] of A
};

struct NetState;

// The dense far block (packed symmetric tiles, eq. (6)) and its tile table, shared by every
// operator built over the same far conductors at the same frequency (several phantoms inside one
// shield): the last operator that holds it frees it. `same` compares the far RWG set (geometry
// and numbering) and the wavenumber.
struct FarShare {
  cxd* z64 = nullptr;
  cxf* z32 = nullptr;
  int* tiles = nullptr;
  int T = 0;
  double k0 = 0;
  std::vector<double> verts;
  std::vector<int> tris, ea, eb, tp, tm;
  bool same(const Rwg& far, double k) const {
    return k == k0 && far.verts == verts && far.tris == tris && far.ea == ea && far.eb == eb && far.tp == tp &&
           far.tm == tm;
  }
  ~FarShare() {
    if (z64) (void)hipFree(z64);
    if (z32) (void)hipFree(z32);
    if (tiles) (void)hipFree(tiles);
  }
};

struct Handle {
  // problem
  int n[3];
  double h, origin[3], freq, omega, k0;
  int nv;
  std::vector<cxd> chi;           // per voxel
  std::vector<int> tissue;        // flat indices
  Rwg far, near;
  RwgDev dfar{}, dnear{};
  int mf = 0, mn = 0;
  int64_t N = 0;
  std::vector<std::vector<PortEdge>> ports;
  // delta-gap tables on the device: the edges of port p are entries [port_off[p], port_off[p + 1])
  // of d_port_idx (global unknown) and d_port_re / d_port_im (value i w eps0 V0 l_m s_m)
  std::vector<int> port_off;
  int* d_port_idx = nullptr;
  double* d_port_re = nullptr;
  double* d_port_im = nullptr;
  vsie_options opts;
  // extended grid
  int ne[3], ob[3], P[3];
  int64_t Ne = 0;
  // pFFT host data
  std::vector<int> base;          // [m_n][3] relative to the body grid
  std::vector<double> Wh;         // [m_n][3][125]
  // grid CSR (by extended-grid voxel)
  int* d_vox2row = nullptr;
  uint8_t* d_rowhasproj = nullptr;   // [ne3][ne2]: x row holds projection voxels
  int* d_rowptr = nullptr;
  int* d_rowrwg = nullptr;
  int n_gridrows = 0;
  int64_t nnz_grid = 0;
  int* d_base = nullptr;          // [m_n][3] in extended-grid coordinates
  // precorrection CSR
  int* d_pc_rowid = nullptr;      // global unknown index of each row
  int* d_pc_rowptr = nullptr;
  int* d_pc_col = nullptr;        // global unknown index
  int n_pcrows = 0;
  int64_t pc_nnz = 0;
  // far block tiling
  int sym_T = 0;
  int* d_tiles = nullptr;         // [ntiles][2] (I, J), I <= J
  std::shared_ptr<FarShare> far_share;   // owner of the dense far block and d_tiles
  uint64_t input_hash = 0;        // inputs that fix the compressed factors (checkpoint key)
  // body mask
  uint8_t* d_mask = nullptr;
  int2* d_runs = nullptr;         // [n3 n2] tissue run of each body x row (see BodyMask)
  int* d_zorder[2] = {};       // z-pass block order, FP64 / FP32, of the candidate in use
  int zcand[2] = {0, 0};       // z-pass candidate chosen by the setup autotuner, FP64 / FP32
  double ztime[2][3] = {};     // its measured time per launch (ms) of every candidate (0: absent)
  // TT
  int tt_r[3][3] = {};
  double tt_err[3] = {0, 0, 0};
  std::vector<cxd> tt_host[3][4];
  // ACA
  int aca_k = 0;
  std::vector<cxd> aca_U, aca_V;
  // generator octant (dimensionless), kept for export and near-field setup
  cxd* d_oct = nullptr;           // [6][ne3][ne2][ne1]
  OpData<double> d64;
  OpData<float> d32;
  bool have32 = false;
  // GMRES workspace (lazily sized)
  // unknowns that couple (conductor currents, tissue voxels), in unknown order: the Krylov vectors
  // hold only these (air voxels carry identity rows and columns and decouple)
  int* d_active = nullptr;
  int64_t n_active = 0;
  cxd* d_full[2] = {};         // full-length product input (zero at air voxels) and output
  cxd* d_krylov = nullptr;
  int64_t krylov_cols = 0;
  cxd* d_solve_work = nullptr;
  double* d_red = nullptr;        // reduction scratch
  cxd* h_pinned = nullptr;        // page-locked host copy of the solver's reductions (HOST_PINNED_ELEMS)
  static constexpr int HOST_PINNED_ELEMS = 2048;
  int64_t device_bytes = 0;
  double setup_seconds = 0;
  // learned preconditioner: material channels of the network, the attached network (applied by
  // the learned solve method) and the network that collects training pairs during solves
  float* d_material = nullptr;   // [n_v][2]
  double mat_scale = 0;
  NetState* net = nullptr;
  NetState* collect = nullptr;
  hipStream_t stream = nullptr;
  std::vector<void*> allocations;
  // per-stage timing of the matrix-vector product (HIP events on the caller's stream)
  static constexpr int NSTAGE = 14;
  hipStream_t side = nullptr;    // second stream of the product (dense far block)
  hipEvent_t fork = nullptr, join = nullptr;
  bool prof = false;
  uint32_t prof_stages = 0;      // stages timed while profiling
  bool concurrent = false;       // far-block chain on the second stream
  // products captured as HIP graphs (vsie_matvec_graph), keyed by precision, columns and buffers
  struct GraphEntry {
    int dtype, nrhs;
    const void* x;
    void* y;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  hipStream_t gstream = nullptr; // capture stream
  // stage events of the last PROF_RING products, read back only by vsie_profile_read (or when the
  // ring wraps), so profiling adds no synchronisation to the products themselves
  static constexpr int PROF_RING = 256;
  hipEvent_t ev[PROF_RING][2 * NSTAGE] = {};
  uint32_t ev_mask[PROF_RING] = {};
  int ring_head = 0, ring_count = 0;
  double prof_ms[NSTAGE] = {};
  int64_t prof_calls[NSTAGE] = {};

  // elimination of the far currents (Schur complement of the dense far block) and the right
  // preconditioner of the reduced system, built on first use
  template <typename R> struct SchurOp {
    cx<R>* S = nullptr;          // L^T Z_ff^-1 L, [K][K]
    cx<R>* ta = nullptr;         // U^T x_n (256)
    cx<R>* pa = nullptr;         // ACA proxies to inject (256)
    cx<R>* p3 = nullptr;         // TT proxies to inject, [3][128]
    cx<R>* Xn = nullptr;         // inverse reduced near block, upper-triangle tiles
    cx<R>* part_n = nullptr;
    cx<R>* invdiag = nullptr;    // inverse body diagonal, 3 n_v (1 for air voxels)
  };
  struct Schur {
    bool ready = false;
    bool precond = false;
    int K = 0;                   // far-coupling proxies: ACA rank + the three TT ranks r3
    DenseLU ff;                  // LU of the dense far block (m_f x m_f, row-major)
    cxd* W = nullptr;            // Z_ff^-1 L, row-major [m_f][K]
    cxd* tc = nullptr;           // compact proxy vector (K)
    cxd* zf = nullptr;           // Z_ff^-1 b_f (m_f)
    cxd* vec[3] = {};            // N-length work vectors of the solver
    int Tn = 0;                  // inverse of the reduced near block as upper-triangle tiles
    int* d_tiles_n = nullptr;
    SchurOp<double> d64;         // per precision: S, proxy buffers, preconditioner
    SchurOp<float> d32;
    double seconds = 0;          // setup time
  } schur;

  template <typename T> T* dalloc(int64_t count) {
    if (count <= 0) count = 1;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, sizeof(T) * (size_t)count);
    if (e != hipSuccess) throw Error(VSIE_E_NOMEM, "hipMalloc of " + std::to_string(sizeof(T) * count) + " bytes failed");
    allocations.push_back(p);
    device_bytes += sizeof(T) * count;
    return (T*)p;
  }
  ~Handle() {
    if (side) (void)hipStreamSynchronize(side);
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    if (gstream) (void)hipStreamDestroy(gstream);
    for (void* p : allocations) (void)hipFree(p);
    if (h_pinned) (void)hipHostFree(h_pinned);
    for (auto& slot : ev)
      for (auto& e : slot)
        if (e) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (side) (void)hipStreamDestroy(side);
  }
};

// host setup (setup_host.cpp)
void build_rwg(const vsie_problem* p, int domain, Rwg& out,
               std::vector<std::pair<int, std::vector<PortEdge>>>& ports);
void stencil_setup(Handle& H);
void fill_gauss_table(GaussTab* t);
void parallel_for(int64_t n, int nthreads, const std::function<void(int64_t, int64_t)>& fn);
int host_threads();   // worker threads for host setup loops (hardware concurrency, at most 16)

// dense host linear algebra (setup_linalg.cpp)
void qr_mgs2(std::vector<cxd>& A, int m, int n, std::vector<cxd>& R);   // A (m x n, row-major) -> Q
std::vector<int> maxvol(const std::vector<cxd>& Q, int m, int r);        // r row indices
bool lu_solve(std::vector<cxd> A, int n, std::vector<cxd>& B, int nrhs);  // A X = B, B (n x nrhs)

// TT-cross and ACA (setup_compress.cpp)
struct EntryFn {
  // evaluate entries of a 4D tensor (i1,i2,i3,i4) for a list of index tuples
  virtual void eval(const std::vector<int>& idx4, std::vector<cxd>& out) = 0;
  virtual ~EntryFn() {}
};
void tt_cross(EntryFn& f, const int n[4], double tol, int rmax, uint64_t seed, std::vector<cxd> cores[4],
              int ranks[3], double* err_est);
// TT rounding of a 4-core train to relative Frobenius accuracy delta (ranks updated in place)
void tt_round(const int n[4], std::vector<cxd> cores[4], int ranks[3], double delta);

}  // namespace vsie
