// extern "C" boundary of the library (declared in include/hinqs.h).
// Each entry point validates its arguments on the host, converts internal
// exceptions into status codes and records the message for hinqs_last_error.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "common.hpp"

using namespace hinqs;

struct hinqs_ctx {
    Ctx c;
};

namespace {

template <typename F>
int guarded(hinqs_ctx *ctx, F &&f) {
    if (!ctx) return HINQS_E_INVALID_ARG;
    ctx->c.err.clear();
    AllocScope scope(&ctx->c.alloc);
    try {
        HQ_CHECK(hipSetDevice(ctx->c.device));
        return f(ctx->c);
    } catch (const Error &e) {
        ctx->c.err = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        ctx->c.err = "host allocation failed";
        return HINQS_E_OOM;
    } catch (const std::exception &e) {
        ctx->c.err = e.what();
        return HINQS_E_HIP;
    }
}

void require_dets(const Ctx &c) {
    if (!c.have_ints) throw Error(HINQS_E_NOT_READY, "integrals are not set");
    if (!c.have_dets) throw Error(HINQS_E_NOT_READY, "determinants are not set");
    if (!c.have_elements) throw Error(HINQS_E_NOT_READY, "matrix elements are not built");
}

void check_sigma_args(const Ctx &c, int k, const void *X, const void *S, int precision) {
    require_dets(c);
    if (!X || !S) throw Error(HINQS_E_INVALID_ARG, "null vector pointer");
    if (k < 1 || k > 16) throw Error(HINQS_E_UNSUPPORTED, "k must be in [1, 16]");
    if (precision != HINQS_FP64 && precision != HINQS_FP32)
        throw Error(HINQS_E_INVALID_ARG, "precision must be HINQS_FP64 or HINQS_FP32");
}

}  // namespace

size_t Ctx::device_bytes() const {
    return d_h.bytes() + d_eri.bytes() + d_eri32.bytes() + sa.bytes() + sb.bytes() + perm.bytes() +
           inv.bytes() + ua.bytes() + ub.bytes() + ga.bytes() + aidx.bytes() + bidx.bytes() +
           gb.bytes() + bperm.bytes() + bm_alpha.bytes() + alink_ptr.bytes() + alink.bytes() +
           alink_info.bytes() + rowptr.bytes() + col.bytes() + desc.bytes() + val.bytes() +
           val32.bytes() + diag.bytes() + diag32.bytes() + work.bytes();
}

extern "C" {

void hinqs_opts_default(hinqs_opts *o) {
    if (!o) return;
    o->block = 8;
    o->max_space = 48;
    o->max_iter = 200;
    o->tol = 1e-8;
    o->precision = HINQS_SOLVE_FP64;
    o->precond_floor = 1e-8;
    o->mixed_switch = 1e-5;
    o->flags = 0;
}

int hinqs_create(hinqs_ctx **out, int device, void *hip_stream, hinqs_alloc_fn alloc_fn,
                 hinqs_free_fn free_fn, void *user) {
    if (!out) return HINQS_E_INVALID_ARG;
    *out = nullptr;
    if ((alloc_fn == nullptr) != (free_fn == nullptr)) return HINQS_E_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HINQS_E_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return HINQS_E_HIP;
    hinqs_ctx *ctx = new (std::nothrow) hinqs_ctx();
    if (!ctx) return HINQS_E_OOM;
    ctx->c.device = device;
    ctx->c.stream = (hipStream_t)hip_stream;
    ctx->c.alloc = Allocator{alloc_fn, free_fn, user, (hipStream_t)hip_stream};
    AllocScope scope(&ctx->c.alloc);
    try {  // sigma row counters: zero here, and put back to zero by every launch
        ctx->c.sigma_ctr.ensure(SIGMA_CTR_WORDS);
    } catch (const Error &) {
        delete ctx;
        return HINQS_E_OOM;
    }
    // on the context's stream: memory from a stream-ordered allocator may still
    // be read by work queued there before it was handed out
    if (hipMemsetAsync(ctx->c.sigma_ctr.p, 0, sizeof(unsigned long long) * SIGMA_CTR_WORDS, ctx->c.stream) !=
            hipSuccess ||
        hipStreamSynchronize(ctx->c.stream) != hipSuccess) {
        delete ctx;
        return HINQS_E_HIP;
    }
    try {  // device address of the static scratch of hinqs_sigma_noalloc (once per device)
        noalloc_setup(device);
    } catch (const Error &e) {
        delete ctx;
        return e.code;
    }
    *out = ctx;
    return HINQS_OK;
}

void hinqs_destroy(hinqs_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->c.device);
    (void)hipStreamSynchronize(ctx->c.stream);
    delete ctx;   // every buffer returns its memory to the allocator it came from
}

const char *hinqs_last_error(const hinqs_ctx *ctx) { return ctx ? ctx->c.err.c_str() : "null context"; }

int hinqs_set_integrals(hinqs_ctx *ctx, int norb, const double *h, const double *eri, double e_core) {
    return guarded(ctx, [&](Ctx &c) {
        if (!h || !eri) throw Error(HINQS_E_INVALID_ARG, "null integral pointer");
        if (norb < 1) throw Error(HINQS_E_INVALID_ARG, "norb must be >= 1");
        if (norb > 32) throw Error(HINQS_E_UNSUPPORTED, "norb > 32 is not supported");
        if (c.have_dets && norb != c.norb)
            throw Error(HINQS_E_INVALID_ARG, "norb differs from that of the determinant set");
        build_integrals(c, norb, h, eri, e_core);
        if (c.have_dets) build_elements(c);
        return HINQS_OK;
    });
}

int hinqs_set_determinants(hinqs_ctx *ctx, int64_t ndet, const uint64_t *alpha, const uint64_t *beta,
                           int nalpha, int nbeta) {
    return guarded(ctx, [&](Ctx &c) {
        if (!c.have_ints) throw Error(HINQS_E_NOT_READY, "set integrals first (they fix norb)");
        if (!alpha || !beta) throw Error(HINQS_E_INVALID_ARG, "null determinant pointer");
        if (ndet < 1 || ndet >= ((int64_t)1 << 31) - 1)
            throw Error(HINQS_E_INVALID_ARG, "ndet must be in [1, 2^31 - 2]");
        if (nalpha < 0 || nbeta < 0 || nalpha > c.norb || nbeta > c.norb)
            throw Error(HINQS_E_INVALID_ARG, "electron counts out of range");
        build_determinants(c, ndet, alpha, beta, nalpha, nbeta, false);
        build_connectivity(c);
        build_elements(c);
        return HINQS_OK;
    });
}

int hinqs_set_determinants_device(hinqs_ctx *ctx, int64_t ndet, const uint64_t *alpha,
                                  const uint64_t *beta, int nalpha, int nbeta) {
    return guarded(ctx, [&](Ctx &c) {
        if (!c.have_ints) throw Error(HINQS_E_NOT_READY, "set integrals first (they fix norb)");
        if (!alpha || !beta) throw Error(HINQS_E_INVALID_ARG, "null determinant pointer");
        if (ndet < 1 || ndet >= ((int64_t)1 << 31) - 1)
            throw Error(HINQS_E_INVALID_ARG, "ndet must be in [1, 2^31 - 2]");
        if (nalpha < 0 || nbeta < 0 || nalpha > c.norb || nbeta > c.norb)
            throw Error(HINQS_E_INVALID_ARG, "electron counts out of range");
        build_determinants(c, ndet, alpha, beta, nalpha, nbeta, true);
        build_connectivity(c);
        build_elements(c);
        return HINQS_OK;
    });
}

int hinqs_sigma(hinqs_ctx *ctx, int k, const void *X, void *S, int precision, int flags) {
    return guarded(ctx, [&](Ctx &c) {
        check_sigma_args(c, k, X, S, precision);
        const int esz = precision == HINQS_FP64 ? 8 : 4;
        const int K = k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : k <= 8 ? 8 : 16;
        const bool sorted = (flags & HINQS_SORTED_ORDER) != 0;
        hipStream_t s = c.stream;
        const bool aligned = ((uintptr_t)X % 16 == 0) && ((uintptr_t)S % 16 == 0);
        if (sorted && K == k && aligned) {
            sigma_sorted(c, K, X, K, S, K, precision, s);
            return HINQS_OK;
        }
        // stage through sorted-order buffers (gather X, scatter S); pad k up to K
        const size_t bytes = (size_t)c.ndet * K * esz;
        sigma_staged(c, k, X, S, precision, sorted, c.cs.get<char>(0, bytes), c.cs.get<char>(1, bytes), nullptr);
        return HINQS_OK;
    });
}

int hinqs_sigma_noalloc(hinqs_ctx *ctx, int k, const void *X, void *S, int precision, int flags) {
    return guarded(ctx, [&](Ctx &c) {
        check_sigma_args(c, k, X, S, precision);
        sigma_noalloc(c, k, X, S, precision, (flags & HINQS_SORTED_ORDER) != 0);
        return HINQS_OK;
    });
}

int hinqs_lowest_eigenpair(hinqs_ctx *ctx, const hinqs_opts *opts, const double *guess, double *energy,
                           double *coeffs, hinqs_stats *stats) {
    return guarded(ctx, [&](Ctx &c) {
        require_dets(c);
        if (!energy || !coeffs) throw Error(HINQS_E_INVALID_ARG, "null output pointer");
        hinqs_opts o;
        hinqs_opts_default(&o);
        if (opts) o = *opts;
        if (!(o.tol > 0) || !(o.precond_floor > 0) || o.max_iter < 1)
            throw Error(HINQS_E_INVALID_ARG, "tol, precond_floor and max_iter must be positive");
        if (o.precision != HINQS_SOLVE_FP64 && o.precision != HINQS_SOLVE_MIXED)
            throw Error(HINQS_E_INVALID_ARG, "unknown precision mode");
        int rc = davidson(c, o, guess, energy, coeffs, stats);
        if (rc == HINQS_E_NOT_CONVERGED) c.err = "Davidson did not reach the tolerance";
        return rc;
    });
}

int hinqs_rdm12(hinqs_ctx *ctx, const double *coeffs, double *rdm1, double *rdm2, int flags) {
    return guarded(ctx, [&](Ctx &c) {
        require_dets(c);
        if (!coeffs || !rdm1 || !rdm2) throw Error(HINQS_E_INVALID_ARG, "null pointer");
        if (flags & HINQS_SORTED_ORDER) {
            rdm12_sorted(c, coeffs, rdm1, rdm2);
        } else {
            double *cs = c.cs.get<double>(0, c.ndet);
            gather_rows(c.stream, coeffs, cs, c.perm.p, c.ndet, 8);
            rdm12_sorted(c, cs, rdm1, rdm2);
        }
        return HINQS_OK;
    });
}

int hinqs_integral_grad(hinqs_ctx *ctx, const double *coeffs, double scale, double *grad_h,
                        double *grad_eri, int flags) {
    return guarded(ctx, [&](Ctx &c) {
        require_dets(c);
        if (!coeffs || !grad_h || !grad_eri) throw Error(HINQS_E_INVALID_ARG, "null pointer");
        if (flags & HINQS_SORTED_ORDER) {
            integral_grad_sorted(c, coeffs, scale, grad_h, grad_eri);
        } else {
            double *cs = c.cs.get<double>(0, c.ndet);
            gather_rows(c.stream, coeffs, cs, c.perm.p, c.ndet, 8);
            integral_grad_sorted(c, cs, scale, grad_h, grad_eri);
        }
        return HINQS_OK;
    });
}

int hinqs_diag(hinqs_ctx *ctx, double *diag, int flags) {
    return guarded(ctx, [&](Ctx &c) {
        require_dets(c);
        if (!diag) throw Error(HINQS_E_INVALID_ARG, "null pointer");
        if (flags & HINQS_SORTED_ORDER)
            HQ_CHECK(hipMemcpyAsync(diag, c.diag.p, 8 * c.ndet, hipMemcpyDeviceToDevice, c.stream));
        else
            scatter_rows(c.stream, c.diag.p, diag, c.perm.p, c.ndet, 8);
        HQ_CHECK(hipStreamSynchronize(c.stream));
        return HINQS_OK;
    });
}

int hinqs_permutation(hinqs_ctx *ctx, int32_t *perm) {
    return guarded(ctx, [&](Ctx &c) {
        if (!c.have_dets) throw Error(HINQS_E_NOT_READY, "determinants are not set");
        if (!perm) throw Error(HINQS_E_INVALID_ARG, "null pointer");
        HQ_CHECK(hipMemcpyAsync(perm, c.perm.p, 4 * c.ndet, hipMemcpyDeviceToDevice, c.stream));
        HQ_CHECK(hipStreamSynchronize(c.stream));
        return HINQS_OK;
    });
}

int hinqs_gram(hinqs_ctx *ctx, int64_t nrows, const double *A, int lda, int ma, const double *B, int ldb,
               int nb, double *G) {
    return guarded(ctx, [&](Ctx &c) {
        if (!A || !B || !G) throw Error(HINQS_E_INVALID_ARG, "null pointer");
        if (nrows < 1 || ma < 1 || nb < 1 || lda < ma || ldb < nb)
            throw Error(HINQS_E_INVALID_ARG, "bad Gram shape");
        if (ma > 96 || nb > 16) throw Error(HINQS_E_UNSUPPORTED, "Gram product limited to 96 x 16");
        gram_product(c, nrows, A, lda, ma, B, ldb, nb, G);
        return HINQS_OK;
    });
}

int hinqs_batch_clear(hinqs_ctx *ctx) {
    return guarded(ctx, [&](Ctx &c) {
        batch_clear(c);
        return HINQS_OK;
    });
}

int hinqs_batch_add(hinqs_ctx *ctx, int norb, const double *h, const double *eri, double e_core, int64_t ndet,
                    const uint64_t *alpha, const uint64_t *beta, int nalpha, int nbeta, int *index) {
    return guarded(ctx, [&](Ctx &c) {
        if (!h || !eri || !alpha || !beta) throw Error(HINQS_E_INVALID_ARG, "null input pointer");
        if (norb < 1) throw Error(HINQS_E_INVALID_ARG, "norb must be >= 1");
        if (norb > 32) throw Error(HINQS_E_UNSUPPORTED, "norb > 32 is not supported");
        if (ndet < 1 || ndet >= ((int64_t)1 << 31) - 1)
            throw Error(HINQS_E_INVALID_ARG, "ndet must be in [1, 2^31 - 2]");
        if (nalpha < 0 || nbeta < 0 || nalpha > norb || nbeta > norb)
            throw Error(HINQS_E_INVALID_ARG, "electron counts out of range");
        const int i = batch_add(c, norb, h, eri, e_core, ndet, alpha, beta, nalpha, nbeta);
        if (index) *index = i;
        return HINQS_OK;
    });
}

int hinqs_batch_info(hinqs_ctx *ctx, int *ninst, int64_t *offsets, int64_t *nnz) {
    return guarded(ctx, [&](Ctx &c) {
        batch_info(c, ninst, offsets, nnz);
        return HINQS_OK;
    });
}

int hinqs_batch_lowest_eigenpair(hinqs_ctx *ctx, const hinqs_opts *opts, double *energies, double *coeffs,
                                 int *status, int *iterations, hinqs_batch_stats *stats) {
    return guarded(ctx, [&](Ctx &c) {
        if (!energies || !coeffs) throw Error(HINQS_E_INVALID_ARG, "null output pointer");
        hinqs_opts o;
        hinqs_opts_default(&o);
        if (opts) o = *opts;
        if (!(o.tol > 0) || !(o.precond_floor > 0) || o.max_iter < 1)
            throw Error(HINQS_E_INVALID_ARG, "tol, precond_floor and max_iter must be positive");
        if (o.precision != HINQS_SOLVE_FP64) throw Error(HINQS_E_UNSUPPORTED, "batched solves run in FP64");
        int rc = batch_solve(c, o, energies, coeffs, status, iterations, stats);
        if (rc == HINQS_E_NOT_CONVERGED) c.err = "some instances did not reach the tolerance";
        return rc;
    });
}

int hinqs_autotune(hinqs_ctx *ctx, int k, int precision, int *shape, double *ms) {
    return guarded(ctx, [&](Ctx &c) {
        require_dets(c);
        if (k != 1 && k != 2 && k != 4 && k != 8 && k != 16)
            throw Error(HINQS_E_UNSUPPORTED, "block size must be 1, 2, 4, 8 or 16");
        const SigmaCfg g = autotune_sigma(c, k, precision);
        if (shape) {
            shape[0] = g.team;
            shape[1] = g.unr;
            shape[2] = g.occ;
        }
        if (ms) *ms = g.ms;
        return HINQS_OK;
    });
}

int hinqs_get_info(hinqs_ctx *ctx, hinqs_info *info) {
    return guarded(ctx, [&](Ctx &c) {
        if (!info) throw Error(HINQS_E_INVALID_ARG, "null pointer");
        info->norb = c.norb;
        info->nalpha = c.na;
        info->nbeta = c.nb;
        info->ndet = c.have_dets ? c.ndet : 0;
        info->nnz = c.have_dets ? c.nnz : 0;
        info->n_alpha_strings = c.nua;
        info->n_beta_strings = c.nub;
        info->device_bytes = (int64_t)c.device_bytes();
        info->ms_sort = c.ms_sort;
        info->ms_connect = c.ms_connect;
        info->ms_elements = c.ms_elements;
        return HINQS_OK;
    });
}

int hinqs_expand(hinqs_ctx *ctx, const double *coeffs, int64_t ntop, int64_t capacity, uint64_t *out_alpha,
                 uint64_t *out_beta, int64_t *count, int32_t *top, int flags) {
    return guarded(ctx, [&](Ctx &c) {
        require_dets(c);
        if (!coeffs || !count) throw Error(HINQS_E_INVALID_ARG, "null pointer");
        if (ntop < 1) throw Error(HINQS_E_INVALID_ARG, "ntop must be at least 1");
        if (capacity < 0 || (capacity > 0 && (!out_alpha || !out_beta)))
            throw Error(HINQS_E_INVALID_ARG, "capacity needs output arrays");
        *count = expand(c, coeffs, (flags & HINQS_SORTED_ORDER) != 0, ntop, capacity, out_alpha, out_beta, top);
        return HINQS_OK;
    });
}

int hinqs_pt2(hinqs_ctx *ctx, const double *coeffs, double e0, int64_t ncand, const uint64_t *cand_alpha,
              const uint64_t *cand_beta, double *numer, double *hxx, double *score, int flags) {
    return guarded(ctx, [&](Ctx &c) {
        require_dets(c);
        if (!coeffs) throw Error(HINQS_E_INVALID_ARG, "null coefficients");
        if (ncand < 0) throw Error(HINQS_E_INVALID_ARG, "ncand must be non-negative");
        if (!std::isfinite(e0)) throw Error(HINQS_E_NONFINITE, "e0 is NaN/Inf");
        if (ncand == 0) return HINQS_OK;
        if (!cand_alpha || !cand_beta) throw Error(HINQS_E_INVALID_ARG, "null candidate strings");
        pt2(c, coeffs, (flags & HINQS_SORTED_ORDER) != 0, e0, ncand, cand_alpha, cand_beta, numer, hxx, score);
        return HINQS_OK;
    });
}

int hinqs_pt2_members(hinqs_ctx *ctx, const double *coeffs, double e0, double *numer, double *hxx, double *score,
                      int flags) {
    return guarded(ctx, [&](Ctx &c) {
        require_dets(c);
        if (!coeffs) throw Error(HINQS_E_INVALID_ARG, "null coefficients");
        if (!std::isfinite(e0)) throw Error(HINQS_E_NONFINITE, "e0 is NaN/Inf");
        pt2_members(c, coeffs, (flags & HINQS_SORTED_ORDER) != 0, e0, numer, hxx, score);
        return HINQS_OK;
    });
}

int hinqs_top_k(hinqs_ctx *ctx, int64_t n, const double *values, int64_t k, int flags, int32_t *idx) {
    return guarded(ctx, [&](Ctx &c) {
        if (!values || !idx) throw Error(HINQS_E_INVALID_ARG, "null pointer");
        if (n < 1 || k < 1 || k > n) throw Error(HINQS_E_INVALID_ARG, "need 1 <= k <= n");
        if (n >= ((int64_t)1 << 31)) throw Error(HINQS_E_UNSUPPORTED, "n must be below 2^31");
        top_k(c, n, values, k, (flags & HINQS_LARGEST) != 0, idx);
        return HINQS_OK;
    });
}

int hinqs_teacher_weights(hinqs_ctx *ctx, const double *coeffs, double *weights, double *p_alpha,
                          double *p_beta, int flags) {
    return guarded(ctx, [&](Ctx &c) {
        if (!c.have_dets) throw Error(HINQS_E_NOT_READY, "determinants are not set");
        if (!coeffs) throw Error(HINQS_E_INVALID_ARG, "null coefficients");
        teacher_weights(c, coeffs, (flags & HINQS_SORTED_ORDER) != 0, weights, p_alpha, p_beta);
        return HINQS_OK;
    });
}

int hinqs_distinct_strings(hinqs_ctx *ctx, uint64_t *alpha, uint64_t *beta) {
    return guarded(ctx, [&](Ctx &c) {
        if (!c.have_dets) throw Error(HINQS_E_NOT_READY, "determinants are not set");
        distinct_strings(c, alpha, beta);
        return HINQS_OK;
    });
}

int hinqs_update_determinants(hinqs_ctx *ctx, int64_t n_evict, const int32_t *evict, int64_t n_add,
                              const uint64_t *add_alpha, const uint64_t *add_beta, const double *coeffs_old,
                              double *coeffs_new, int flags, double *ms) {
    return guarded(ctx, [&](Ctx &c) {
        require_dets(c);
        if (n_evict < 0 || n_add < 0) throw Error(HINQS_E_INVALID_ARG, "negative count");
        if (n_evict > 0 && !evict) throw Error(HINQS_E_INVALID_ARG, "null evict list");
        if (n_add > 0 && (!add_alpha || !add_beta)) throw Error(HINQS_E_INVALID_ARG, "null appended strings");
        if ((coeffs_old == nullptr) != (coeffs_new == nullptr))
            throw Error(HINQS_E_INVALID_ARG, "coeffs_old and coeffs_new go together");
        if (n_evict > c.ndet) throw Error(HINQS_E_INVALID_ARG, "more evictions than determinants");
        update_determinants(c, n_evict, evict, n_add, add_alpha, add_beta, coeffs_old, coeffs_new,
                            (flags & HINQS_SORTED_ORDER) != 0, ms);
        return HINQS_OK;
    });
}

int hinqs_grow_basis(hinqs_ctx *ctx, int mode, int64_t ncand, const uint64_t *cand_alpha, const uint64_t *cand_beta,
                     const double *cand_score, int64_t k, const double *basis_score, int64_t b_max,
                     const double *coeffs_old, double *coeffs_new, double *score_new, int64_t *ndet_new, double *ms) {
    return guarded(ctx, [&](Ctx &c) {
        require_dets(c);
        if (mode != HINQS_GROW_APPEND && mode != HINQS_GROW_REBUILD)
            throw Error(HINQS_E_INVALID_ARG, "unknown mode");
        if (ncand < 0 || k < 0 || b_max < 0) throw Error(HINQS_E_INVALID_ARG, "negative size");
        if (ncand > 0 && (!cand_alpha || !cand_beta || !cand_score))
            throw Error(HINQS_E_INVALID_ARG, "null candidate arrays");
        const bool capped = mode == HINQS_GROW_APPEND && b_max > 0 && c.ndet + std::min(k, ncand) > b_max;
        if (!basis_score && (mode == HINQS_GROW_REBUILD || capped || score_new))
            throw Error(HINQS_E_INVALID_ARG, "basis_score is required");
        if ((coeffs_old == nullptr) != (coeffs_new == nullptr))
            throw Error(HINQS_E_INVALID_ARG, "coeffs_old and coeffs_new go together");
        if (c.ndet + ncand >= ((int64_t)1 << 31)) throw Error(HINQS_E_UNSUPPORTED, "too many entries");
        const int64_t n = grow_basis(c, mode, ncand, cand_alpha, cand_beta, cand_score, k, basis_score, b_max,
                                     coeffs_old, coeffs_new, score_new, ms);
        if (ndet_new) *ndet_new = n;
        return HINQS_OK;
    });
}

int hinqs_get_determinants(hinqs_ctx *ctx, uint64_t *alpha, uint64_t *beta) {
    return guarded(ctx, [&](Ctx &c) {
        if (!c.have_dets) throw Error(HINQS_E_NOT_READY, "determinants are not set");
        caller_strings(c, alpha, beta);
        return HINQS_OK;
    });
}

int hinqs_product_closure(hinqs_ctx *ctx, int64_t capacity, uint64_t *out_alpha, uint64_t *out_beta,
                          int64_t *count) {
    return guarded(ctx, [&](Ctx &c) {
        if (!c.have_dets) throw Error(HINQS_E_NOT_READY, "determinants are not set");
        if (!count) throw Error(HINQS_E_INVALID_ARG, "null count");
        if (capacity < 0 || (capacity > 0 && (!out_alpha || !out_beta)))
            throw Error(HINQS_E_INVALID_ARG, "capacity needs output arrays");
        *count = product_closure(c, capacity, out_alpha, out_beta);
        return HINQS_OK;
    });
}

uint32_t hinqs_pair_descriptor(uint64_t alpha_i, uint64_t beta_i, uint64_t alpha_j, uint64_t beta_j) {
    return pair_desc((uint32_t)alpha_i, (uint32_t)beta_i, (uint32_t)alpha_j, (uint32_t)beta_j);
}

int hinqs_connectivity(hinqs_ctx *ctx, int64_t *rowptr, int32_t *col, uint32_t *desc) {
    return guarded(ctx, [&](Ctx &c) {
        if (!c.have_dets) throw Error(HINQS_E_NOT_READY, "determinants are not set");
        if (!rowptr) throw Error(HINQS_E_INVALID_ARG, "null rowptr");
        export_connectivity(c, rowptr, col, desc);
        return HINQS_OK;
    });
}

}  // extern "C"
