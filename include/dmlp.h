/*
 * dmlp.h -- C ABI of the emittance surrogate on one AMD MI355X (gfx950):
 * a multilayer perceptron from the 7 lattice parameters and the 6 initial
 * beam sizes to the final x and y emittances, evaluated together with its
 * 2 x 13 input Jacobian, and trained with a Sobolev loss on values and
 * gradients produced by the differentiable PIC library (dpic.h).
 *
 * The network (13 -> 256 -> 256 -> 256 -> 256 -> 2, SiLU on the hidden
 * layers) runs on the matrix cores in BF16 with FP32 accumulation. Each
 * sample travels as 16 columns: the activation and its 13 tangents (the
 * forward-mode derivatives with respect to the normalised inputs, as in the
 * dual-number rules of Sec. 2) plus 2 zero columns, so every layer is one
 * dense product W [out x in] times [in x 16 n]. Hidden activations and the
 * backward products are stored in BF16; the master weights, the Adam
 * moments, the loss and all outputs are FP32/FP64.
 *
 * Normalisation: u = (x - in_center) / in_scale enters the network, and
 * eps = out_center + out_scale * o leaves it; returned Jacobians are
 * d eps / d x.
 *
 * Sobolev loss over n samples with targets (eps_t, jac_t), in normalised
 * units:  loss = (1/n) sum_s [ wv |o_s - y_s|^2 + wj |J_s - G_s|_F^2 ],
 * y = (eps_t - out_center) / out_scale, G = jac_t * in_scale / out_scale.
 *
 * Parameter vector (FP32, packed): W1 [256][13], b1 [256], W2 [256][256],
 * b2, W3, b3, W4, b4, W5 [2][256], b5 [2]  (W row-major [out][in]).
 *
 * Conventions as in dpic.h: int return codes (DPIC_OK / DPIC_E*), *_dev are
 * device pointers, the caller owns the device workspace, work is enqueued on
 * the stream bound at creation, calls returning host data synchronise.
 */
#ifndef DMLP_H
#define DMLP_H

#include <stddef.h>
#include <stdint.h>

#include "dpic.h"

#ifdef __cplusplus
extern "C" {
#endif

#define DMLP_NIN 13
#define DMLP_NOUT 2
#define DMLP_HIDDEN 256
#define DMLP_LAYERS 5

typedef struct dmlp_ctx dmlp_ctx;

/* Number of FP32 parameters in the packed vector (201474). */
int dmlp_param_count(void);

/* Device workspace bytes for batches of up to nmax samples. */
int dmlp_query_workspace(int nmax, size_t* bytes);

/* Bind caller-owned workspace (256-byte aligned) and a stream. */
int dmlp_create(int nmax, void* workspace_dev, size_t workspace_bytes, void* hip_stream, dmlp_ctx** out);
int dmlp_destroy(dmlp_ctx* ctx);
int dmlp_last_error(const dmlp_ctx* ctx, char* buf, size_t len);

/* in_center[13], in_scale[13] (> 0), out_center[2], out_scale[2] (> 0). */
int dmlp_set_normalization(dmlp_ctx* ctx, const double* in_center, const double* in_scale, const double* out_center,
                           const double* out_scale);

/* Copy the packed FP32 parameters in (resets the Adam moments) or out. Synchronous. */
int dmlp_set_params(dmlp_ctx* ctx, const float* params);
int dmlp_get_params(dmlp_ctx* ctx, float* params);

/*
 * Inference on n <= nmax samples: x_dev [n][13] -> eps_dev [n][2] and, if
 * not NULL, jac_dev [n][2][13] = d eps / d x (FP64, device). Asynchronous.
 */
int dmlp_predict(dmlp_ctx* ctx, int n, const double* x_dev, double* eps_dev, double* jac_dev);

/*
 * Loss and its gradient with respect to the packed parameters for the
 * samples (x_dev [n][13], targets eps_dev [n][2], jac_dev [n][2][13]).
 * loss (host) and grad (host, dmlp_param_count() floats) may be NULL.
 * Synchronous; the parameters are not changed.
 */
int dmlp_loss_grad(dmlp_ctx* ctx, int n, const double* x_dev, const double* eps_dev, const double* jac_dev,
                   double wv, double wj, double* loss, float* grad);

/*
 * One Adam step (learning rate lr; moments from dmlp_set_adam, default
 * 0.9, 0.999, 1e-8) on the loss of this batch. Asynchronous; the batch loss
 * is kept on the device (dmlp_read_loss).
 */
int dmlp_train_step(dmlp_ctx* ctx, int n, const double* x_dev, const double* eps_dev, const double* jac_dev,
                    double wv, double wj, double lr);
int dmlp_set_adam(dmlp_ctx* ctx, double beta1, double beta2, double eps);
int dmlp_read_loss(dmlp_ctx* ctx, double* loss);

#ifdef __cplusplus
}
#endif
#endif /* DMLP_H */
