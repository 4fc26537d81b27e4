// capi.hip -- host-side entry points of the C ABI: space validation, id
// decoding, status strings.
#include "common.hpp"

using namespace sisso;

extern "C" sisso_status sisso_space_init(sisso_space *s)
{
    if (!s) return SISSO_E_NULL;
    if (s->d < 1 || s->levels < 1 || s->levels > SISSO_MAX_LEVELS || s->rect < 0 || s->rect > 2)
        return SISSO_E_SHAPE;
    if (s->n_unary < 0 || s->n_unary > SISSO_MAX_UNARY || s->n_binary < 0 || s->n_binary > SISSO_MAX_BINARY)
        return SISSO_E_SHAPE;
    unsigned seen = 0;
    for (int i = 0; i < s->n_unary; ++i) {
        const int op = s->unary[i];
        if (op < SISSO_SQ || op > SISSO_SIN || (seen >> op) & 1u) return SISSO_E_SHAPE;
        seen |= 1u << op;
    }
    for (int i = 0; i < s->n_binary; ++i) {
        const int op = s->binary[i];
        if (op < SISSO_ADD || op > SISSO_DIV || (seen >> op) & 1u) return SISSO_E_SHAPE;
        seen |= 1u << op;
    }
    s->n_slots = 0;
    for (int i = 0; i < 2 * SISSO_MAX_BINARY; ++i) { s->slot_op[i] = -1; s->slot_rev[i] = 0; }
    for (int i = 0; i < s->n_binary; ++i) {
        s->slot_op[s->n_slots] = s->binary[i];
        s->slot_rev[s->n_slots] = 0;
        s->n_slots++;
        if (s->binary[i] == SISSO_DIV) {
            s->slot_op[s->n_slots] = SISSO_DIV;
            s->slot_rev[s->n_slots] = 1;
            s->n_slots++;
        }
    }
    // level sizes (|P_l| = |P_{l-1}| + U |N_{l-1}| + S (C(p_{l-1}, 2) - C(p_{l-2}, 2)))
    const double lim = 4.0e18;
    int64_t prev2 = 0, prev = s->d;
    for (int l = 0; l <= SISSO_MAX_LEVELS; ++l) s->pool[l] = 0;
    s->pool[0] = s->d;
    for (int l = 1; l <= s->levels; ++l) {
        const double sz = (double)prev + (double)s->n_unary * (double)(prev - prev2) +
                          (double)s->n_slots * ((double)choose2(prev) - (double)choose2(prev2));
        if (sz > lim) return SISSO_E_RANGE;
        const int64_t size = prev + (int64_t)s->n_unary * (prev - prev2) +
                             (int64_t)s->n_slots * (choose2(prev) - choose2(prev2));
        s->pool[l] = size;
        prev2 = prev;
        prev = size;
    }
    for (int l = s->levels + 1; l <= SISSO_MAX_LEVELS; ++l) s->pool[l] = s->pool[s->levels];
    s->total = s->pool[s->levels];
    s->rect_unary = s->rect_binary = 0;
    if (s->rect) {
        // rect 1: the one-sided slice (u new at level L, v in P_{L-1});
        // rect 2: the whole next TRI level (u new at level L, v < u)
        const int64_t lo = s->pool[s->levels - 1], hi = s->pool[s->levels];
        const int64_t nlast = hi - lo;
        const double pairs = s->rect == 1 ? (double)nlast * (double)lo : (double)choose2(hi) - (double)choose2(lo);
        const double sz = (double)s->total + (double)s->n_unary * nlast + (double)s->n_slots * pairs;
        if (sz > lim) return SISSO_E_RANGE;
        s->rect_unary = (int64_t)s->n_unary * nlast;
        s->rect_binary = (int64_t)s->n_slots * (s->rect == 1 ? nlast * lo : choose2(hi) - choose2(lo));
        s->total += s->rect_unary + s->rect_binary;
    }
    if (s->total < 1) return SISSO_E_SHAPE;
    return SISSO_OK;
}

extern "C" sisso_status sisso_decode(const sisso_space *space, int64_t id, int32_t *op, int64_t *left,
                                     int64_t *right)
{
    if (!space || !op || !left || !right) return SISSO_E_NULL;
    int o;
    int64_t l, r;
    if (decode_id(*space, id, &o, &l, &r)) return SISSO_E_RANGE;
    *op = o;
    *left = l;
    *right = r;
    return SISSO_OK;
}

extern "C" const char *sisso_status_string(sisso_status st)
{
    switch (st) {
    case SISSO_OK: return "ok";
    case SISSO_E_NULL: return "null pointer argument";
    case SISSO_E_SHAPE: return "size or leading dimension out of range";
    case SISSO_E_RANGE: return "id, range or k outside the space";
    case SISSO_E_WORKSPACE: return "workspace too small";
    case SISSO_E_UNSUPPORTED: return "unsupported request";
    case SISSO_E_DEVICE: return "HIP runtime error";
    case SISSO_E_NUMERIC: return "numerical degeneracy";
    default: return "unknown status";
    }
}

extern "C" const char *sisso_version(void) { return "sisso-mi355x 0.1 (gfx950)"; }
