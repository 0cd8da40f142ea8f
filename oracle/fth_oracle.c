/*
 * FP64 CPU oracle for the f-thermostat (FTH) time stepping.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library or its Python binding may
 * link, load or call this file; only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark do.  It shares no code with the HIP path.
 *
 * What it computes (Nava, Ceriotti, Dryzun, Parrinello, "Evaluating functions
 * of positive-definite matrices using colored noise thermostats"):
 *
 *   - the harmonic potential V = q^T M q / 2 of Sec. I (Eq. for V(q)), whose
 *     force is F = -M q (dense rows or CSR rows, summed in stored order);
 *   - the Markovian GLE of Sec. I (extended-momentum SDE, drift A_p and
 *     diffusion B_p, free-particle covariance C_p) applied independently to
 *     every Cartesian degree of freedom, integrated as an exact
 *     Ornstein-Uhlenbeck step (p, s) <- T (p, s) + S xi with T = exp(-A_p h)
 *     and S S^T = C_p - T C_p T^T, placed between the two half kicks of a
 *     velocity-Verlet step (the "modified velocity Verlet" the paper cites);
 *   - the time averages <q_i q_j> of Sec. I (the covariance estimator of the
 *     normal-mode argument) accumulated in FP64 with block averaging
 *     (Sec. II, memory-footprint paragraph: "collect and block-average").
 *
 * T and S arrive as inputs (computed by the Python side of the oracle with
 * library routines), so this file only holds the step loop and the noise.
 *
 * Noise: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from that
 * paper's definition; Box-Muller on the resulting uniforms.  The counter layout
 * is this project's: for degree of freedom i, replica r, step n, noise
 * component j and stream sigma the counter is
 *     (i mod 2^32, n mod 2^32, (j << 16) | (r >> 2), sigma),
 * the key is (seed mod 2^32, seed >> 32), word (r & 3) of the block is used,
 * words are mapped to u = (2*(x >> 9) + 1) * 2^-24 in (0, 1), and the pairs
 * (u0, u1), (u2, u3) go through Box-Muller (cos for the even word, sin for the
 * odd word).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- Philox */
/* Multipliers and Weyl key increments of Philox4x32 (SC'11, Table 2). */
static const uint32_t PH_M0 = 0xD2511F53u;
static const uint32_t PH_M1 = 0xCD9E8D57u;
static const uint32_t PH_W0 = 0x9E3779B9u;
static const uint32_t PH_W1 = 0xBB67AE85u;

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += PH_W0; k1 += PH_W1; }
        uint64_t prod0 = (uint64_t)PH_M0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)PH_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double orc_u01(uint32_t x)
{
    return (2.0 * (double)(x >> 9) + 1.0) * 0x1p-24;
}

/* Four normals of one Philox block: replicas 4*quad .. 4*quad+3 of noise
 * component j for dof i at step n. */
void orc_noise_block(uint64_t seed, uint32_t stream, uint64_t i, uint64_t n,
                     uint32_t j, uint32_t quad, double z[4])
{
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)n, (j << 16) | (quad & 0xFFFFu), stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    const double two_pi = 6.283185307179586476925286766559;
    double u0 = orc_u01(x[0]), u1 = orc_u01(x[1]), u2 = orc_u01(x[2]), u3 = orc_u01(x[3]);
    double ra = sqrt(-2.0 * log(u0));
    double rb = sqrt(-2.0 * log(u2));
    z[0] = ra * cos(two_pi * u1);
    z[1] = ra * sin(two_pi * u1);
    z[2] = rb * cos(two_pi * u3);
    z[3] = rb * sin(two_pi * u3);
}

double orc_normal(uint64_t seed, uint32_t stream, uint64_t i, uint32_t r, uint64_t n, uint32_t j)
{
    double z[4];
    orc_noise_block(seed, stream, i, n, j, r >> 2, z);
    return z[r & 3u];
}

/* Batch form for tests: out[k] = normal(seed, stream, i[k], r[k], n[k], j[k]). */
void orc_normals(uint64_t seed, uint32_t stream, int64_t count, const uint64_t* i,
                 const uint32_t* r, const uint64_t* n, const uint32_t* j, double* out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < count; ++k)
        out[k] = orc_normal(seed, stream, i[k], r[k], n[k], j[k]);
}

void orc_philox_batch(int64_t count, const uint32_t* ctr, const uint32_t* key, uint32_t* out)
{
    for (int64_t k = 0; k < count; ++k)
        orc_philox4x32_10(ctr + 4 * k, key, out + 4 * k);
}

/* ------------------------------------------------------------ integrator */
/*
 * Advances the state by nsteps steps starting at global step index n0.
 *
 * Matrix: fmt == 0 -> dense row-major dense[N*N]; fmt == 1 -> CSR
 * (row_ptr[N+1], col[nnz], val[nnz]).
 * Propagator: T, S are (ns+1)x(ns+1) row-major.
 * State: q[i*R + r], p[i*R + r], s[(k*N + i)*R + r] for k = 0..ns-1.
 * Accumulators (one per pair, pairs[2*k], pairs[2*k+1]):
 *   blk  = sum of x over the current (incomplete) block,
 *   s1   = sum over completed blocks of the block sums,
 *   s2   = sum over completed blocks of the squared block sums,
 * where x(n) = sum_r q_i^r(n) q_j^r(n) for every n >= burn_in, or, by kinds[k]:
 *   1: the momentum form sum_r p_i^r(n) p_j^r(n) of Eq. 7 (p_n, the momentum
 *      at the start of step n, the same instant as q_n);
 *   2: the trace sum_i sum_r q_i^r(n)^2 (Tr of the position response);
 *   3: sum_i sum_r q_i^r(n) (M q(n))_i^r, i.e. q^T M q = -q . F, the trace
 *      Tr[O g(M)] with O = M (Sec. I, traces of the form Tr O f(M));
 *   4: the kinetic trace sum_i sum_r p_i^r(n)^2 (Tr f(M) of Sec. I);
 * the pair indices of kinds 2-4 are ignored.  kinds may be NULL (all
 * position pairs).  A block closes after the step with
 * (n - burn_in + 1) % L == 0 and then *nblocks grows by one.
 *
 * One step n (all dofs and replicas):
 *   1. F = -M q_n
 *   2. accumulate x(n) from q_n (or p_n)
 *   3. p += (h/2) F
 *   4. (p, s) <- T (p, s) + S xi(n)
 *   5. p += (h/2) F
 *   6. q_{n+1} = q_n + h p
 * Returns 0, or -1 on allocation failure.
 */
int orc_run(int64_t N, int fmt, const double* dense, const int64_t* row_ptr,
            const int32_t* col, const double* val, int ns, const double* T,
            const double* S, double h, int64_t R, uint64_t seed, uint32_t stream,
            int64_t n0, int64_t nsteps, int64_t burn_in, int64_t L, double* q,
            double* p, double* s, int64_t npairs, const int32_t* pairs, const int32_t* kinds, double* blk,
            double* s1, double* s2, int64_t* nblocks, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const int D = ns + 1;
    /* threads only pay off on large systems */
    const int par = (N * R) >= 16384;
    double* F = (double*)malloc(sizeof(double) * (size_t)(N * R));
    double* qn = (double*)malloc(sizeof(double) * (size_t)(N * R));
    if (!F || !qn) { free(F); free(qn); return -1; }

    for (int64_t step = 0; step < nsteps; ++step) {
        const int64_t n = n0 + step;

        /* 1. force from q_n */
        #pragma omp parallel for schedule(static) if(par)
        for (int64_t i = 0; i < N; ++i) {
            for (int64_t r = 0; r < R; ++r) {
                double acc = 0.0;
                if (fmt == 0) {
                    for (int64_t j = 0; j < N; ++j)
                        acc += dense[i * N + j] * q[j * R + r];
                } else {
                    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
                        acc += val[k] * q[(int64_t)col[k] * R + r];
                }
                F[i * R + r] = -acc;
            }
        }

        /* 2. accumulate <q_i q_j> from q_n (<p_i p_j> from p_n) */
        if (n >= burn_in && npairs > 0) {
            const int close = ((n - burn_in + 1) % L) == 0;
            #pragma omp parallel for schedule(static) if(npairs * R >= 16384)
            for (int64_t k = 0; k < npairs; ++k) {
                const int kind = kinds ? kinds[k] : 0;
                double x = 0.0;
                if (kind <= 1) {
                    const int64_t a = pairs[2 * k], b = pairs[2 * k + 1];
                    const double* v = kind == 1 ? p : q;
                    for (int64_t r = 0; r < R; ++r)
                        x += v[a * R + r] * v[b * R + r];
                } else {
                    for (int64_t i = 0; i < N * R; ++i)
                        x += kind == 2 ? q[i] * q[i] : kind == 3 ? -q[i] * F[i] : p[i] * p[i];
                }
                blk[k] += x;
                if (close) {
                    s1[k] += blk[k];
                    s2[k] += blk[k] * blk[k];
                    blk[k] = 0.0;
                }
            }
            if (close) *nblocks += 1;
        }

        /* 3-6. kick, GLE O-step, kick, drift */
        #pragma omp parallel for schedule(static) if(par)
        for (int64_t i = 0; i < N; ++i) {
            double x[64], y[64], xi[64];
            for (int64_t r = 0; r < R; ++r) {
                const double f = F[i * R + r];
                x[0] = p[i * R + r] + 0.5 * h * f;
                for (int k = 0; k < ns; ++k)
                    x[k + 1] = s[((int64_t)k * N + i) * R + r];
                for (int j = 0; j < D; ++j)
                    xi[j] = orc_normal(seed, stream, (uint64_t)i, (uint32_t)r, (uint64_t)n, (uint32_t)j);
                for (int a = 0; a < D; ++a) {
                    double v = 0.0;
                    for (int b = 0; b < D; ++b) v += T[a * D + b] * x[b];
                    for (int b = 0; b < D; ++b) v += S[a * D + b] * xi[b];
                    y[a] = v;
                }
                const double pn = y[0] + 0.5 * h * f;
                p[i * R + r] = pn;
                for (int k = 0; k < ns; ++k)
                    s[((int64_t)k * N + i) * R + r] = y[k + 1];
                qn[i * R + r] = q[i * R + r] + h * pn;
            }
        }
        memcpy(q, qn, sizeof(double) * (size_t)(N * R));
    }
    free(F);
    free(qn);
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
